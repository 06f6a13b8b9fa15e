"""Failure handling of the GPU path with batched replicas: a non-finite value in one
replica leaves the other replicas' results bit for bit as without it, and a coupled step
that meets it returns HSF_ENONFINITE with the whole context as at the step's start.

Every kernel still exits normally: the non-finite values are ordinary inputs (NaN fields,
densities or LB populations set from the host), detected by the library's own checks.
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


BOXES = [(12, 10, 9), (16, 16, 16), (9, 11, 13)]


def batch(precision):
    return [W.Workload(f"rep{i}", L, W.chain(3, 5), False, W.chi_matrix(ab=(18.0 + 2 * i) / 8), tau=1.0,
                       noise=0.01, seed=i, precision=precision) for i, L in enumerate(BOXES)]


def slices(ctx, wls, per_site):
    """Per replica: slice of a concatenated array with per_site values per site."""
    return [slice(per_site * ctx.site_offset(r), per_site * ctx.site_offset(r) + per_site * wl.V)
            for r, wl in enumerate(wls)]


def state(ctx):
    return ctx.get_densities(), ctx.get_fields(), ctx.get_lb()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nan_replica_leaves_the_others(hsf, precision):
    """A NaN field in replica 1: the evaluation returns HSF_ENONFINITE, and the densities
    and Q of replicas 0 and 2 equal, bit for bit, those of the same fields with replica 1
    finite."""
    say(f"[failure] nan field, 3 replicas, {precision}")
    wls = batch(precision)
    tol = 1e-9 if precision == "fp64" else 1e-6
    ctx = hsf.Context(wls)
    ctx.set_densities(np.concatenate([W.initial_composition(w).ravel() for w in wls]))
    ctx.step(3, tol=tol, max_iter=2000)
    fs = slices(ctx, wls, ctx.nsp)
    w_good = ctx.get_fields()
    ref = np.empty(ctx.nsp * ctx.T)
    _, q_ref = ctx.evaluate(out=ref)
    w_bad = w_good.copy()
    w_bad[fs[1].start + wls[1].V // 3] = np.nan
    ctx.set_fields(w_bad)
    got = np.full(ctx.nsp * ctx.T, -1.0)
    with pytest.raises(hsf.HsfError) as ei:
        ctx.evaluate(out=got)
    assert ei.value.code == hsf.HSF_ENONFINITE
    for r in (0, 2):
        assert np.array_equal(got[fs[r]], ref[fs[r]]), r
    assert not np.all(np.isfinite(got[fs[1]]))
    ctx.set_fields(w_good)
    got2, q2 = ctx.evaluate()
    assert np.array_equal(got2, ref) and np.array_equal(q2, q_ref)
    ctx.close()


@pytest.mark.parametrize("where", ["density", "lb"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nonfinite_step_rolls_back(hsf, precision, where):
    """A NaN density (met by the inversion) or a NaN LB population (met by the LB step,
    after the inversion has converged) in replica 1: hsf_step returns HSF_ENONFINITE after
    the steps before it, and the context holds exactly the state of the failing step's
    start, every replica included.  With the finite value put back, the run continues bit
    for bit like a run that never met it."""
    say(f"[failure] rollback, nan {where}, {precision}")
    wls = batch(precision)
    tol = 1e-9 if precision == "fp64" else 1e-6
    phi0 = np.concatenate([W.initial_composition(w).ravel() for w in wls])

    def fresh():
        c = hsf.Context(wls)
        c.set_densities(phi0)
        c.set_warm(hsf.WARM_EXTRAP)
        c.step(3, tol=tol, max_iter=2000)
        return c

    ref = fresh()
    ref.step(2, tol=tol, max_iter=2000)
    ref_state = state(ref)
    ctx = fresh()
    start = state(ctx)
    if where == "density":
        bad = start[0].copy()
        bad[slices(ctx, wls, ctx.nsp)[1].start + 7] = np.nan
        ctx.set_densities(bad)
    else:
        bad = start[2].copy()
        bad[slices(ctx, wls, 19)[1].start + 5 * wls[1].V + 11] = np.nan
        ctx.set_lb(bad)
    before = state(ctx)
    with pytest.raises(hsf.HsfError) as ei:
        ctx.step(2, tol=tol, max_iter=2000)
    assert ei.value.code == hsf.HSF_ENONFINITE
    after = state(ctx)
    for a, b in zip(after, before):
        assert np.array_equal(a, b, equal_nan=True)
    # put the finite value back: the same two steps as the reference run
    ctx.set_densities(start[0])
    ctx.set_lb(start[2])
    ctx.step(2, tol=tol, max_iter=2000)
    for a, b in zip(state(ctx), ref_state):
        assert np.array_equal(a, b)
    ctx.close()
    ref.close()


def test_unstable_time_step_is_reported(hsf):
    """A time step far above the explicit scheme's stability limit (dt = 0.25 against a
    limit of about 0.015 for kappa = 10): the composition's short-wavelength modes grow
    every step until a step's inversion can no longer reach its targets; hsf_step then
    reports the failure (HSF_ENOCONV or HSF_ENONFINITE) with the densities of that step's
    start.  The same run at dt = 0.01 takes every step."""
    wl = W.melt16_a4b4().with_(L=(12, 12, 12))
    fails = None
    for dt, steps in ((0.01, 40), (0.25, 40)):
        ctx = hsf.Context(wl.with_(dt=dt))
        ctx.set_densities(W.initial_composition(wl).ravel())
        for k in range(steps):
            before = ctx.get_densities()
            try:
                ctx.step(1, tol=1e-8, max_iter=300)
            except hsf.HsfError as e:
                assert dt == 0.25, (dt, k, e)
                assert e.code in (hsf.HSF_ENOCONV, hsf.HSF_ENONFINITE)
                fails = (k, e.code, float(np.abs(before - before.mean()).max()))
                assert np.array_equal(ctx.get_densities(), before)
                break
        say(f"[unstable dt] dt {dt}: {'failure at step %d (code %d, max |dphi| %.3g)' % fails if dt == 0.25 else 'all steps taken'}")
        ctx.close()
    assert fails is not None, "the unstable run took every step"
