"""The step log (hsf_set_step_log / hsf_read_step_log): one record per replica and
successful coupled step, whose figures equal what the context reports through its other
entry points, and which leaves the run bit for bit as without it."""
import json
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


def batch(hydro):
    """Two uneven solutions of one chain (a context holds one chain architecture)."""
    return [W.Workload("solution", (12, 10, 9), W.chain(2, 6), True, W.chi_matrix(ab=20 / 8, bs=28 / 8), tau=1.0,
                       noise=0.01, seed=1, phi_p=0.3, hydro=hydro),
            W.Workload("solution", (9, 11, 13), W.chain(2, 6), True, W.chi_matrix(ab=22 / 8, bs=30 / 8), tau=0.8,
                       noise=0.01, seed=2, phi_p=0.2, hydro=hydro)]


def run(hsf, wls, steps, log):
    ctx = hsf.Context(wls)
    ctx.set_densities(np.concatenate([W.initial_composition(w).ravel() for w in wls]))
    if log:
        ctx.set_step_log(True)
    stats = None
    for _ in range(steps):
        stats, _ = ctx.step(1, tol=1e-9, max_iter=2000)
    return ctx, stats


@pytest.mark.parametrize("hydro", [True, False])
def test_step_log_records(hsf, hydro, tmp_path):
    """Five steps of two uneven replicas (solutions of different boxes and chi): ten
    records in step order; the last step's iteration and evaluation counts, residual and
    convergence equal hsf_step's statistics; the amounts equal the site sums of the
    densities after the step (1e-12 relative); max |u| equals the largest speed of
    hsf_get_flow's velocity (0 with the flow off); ln Q equals that of an evaluation at
    the step's converged fields (1e-10); the phase times are positive.  The densities and
    fields equal, bit for bit, those of the same run without the log."""
    say(f"[step log] hydro {hydro}")
    wls = batch(hydro)
    ctx, stats = run(hsf, wls, 5, True)
    recs = ctx.read_step_log()
    assert len(recs) == 10
    assert [(r["step"], r["replica"]) for r in recs] == [(s, q) for s in range(1, 6) for q in range(2)]
    phi = ctx.get_densities()
    _, u = ctx.get_flow()
    _, q = ctx.evaluate()
    for r, wl in enumerate(wls):
        rec = recs[8 + r]
        assert rec["iterations"] == stats[r]["iterations"]
        assert rec["evaluations"] == stats[r]["evaluations"]
        assert rec["converged"] == 1 and rec["residual"] == stats[r]["residual"]
        fo = ctx.field_offset(r)
        p = phi[fo:fo + wl.nsp * wl.V].reshape(wl.nsp, -1)
        for I in range(3):
            want = p[I].sum()
            assert abs(rec["amount"][I] - want) <= 1e-12 * max(1.0, abs(want)), (r, I)
        so = ctx.site_offset(r)
        if hydro:
            uu = u[3 * so:3 * so + 3 * wl.V].reshape(3, -1)
            want_u = float(np.sqrt((uu ** 2).sum(0)).max())
            assert want_u > 0 and abs(rec["max_u"] - want_u) <= 1e-12 * want_u
        else:
            assert rec["max_u"] == 0.0
        assert abs(rec["ln_q"] - np.log(q[r])) <= 1e-10
        assert rec["ms_inversion"] > 0 and rec["ms_dynamics"] > 0
    say(f"  last records: {recs[-2:]}")
    assert ctx.read_step_log() == []
    ref, _ = run(hsf, wls, 5, False)
    assert np.array_equal(ref.get_densities(), phi) and np.array_equal(ref.get_fields(), ctx.get_fields())
    # JSON lines
    ctx.step(2, tol=1e-9, max_iter=2000)
    path = tmp_path / "steps.jsonl"
    assert ctx.write_step_log(str(path)) == 4
    lines = [json.loads(ln) for ln in path.read_text().splitlines()]
    assert [ln["step"] for ln in lines] == [6, 6, 7, 7]
    ctx.close()
    ref.close()


def test_step_log_skips_failed_steps_and_stops(hsf):
    """A step that meets a NaN density returns HSF_ENONFINITE and adds no record; the next
    successful step is numbered after the last successful one; switching the log off drops
    the unread records and records nothing more."""
    wls = batch(True)
    ctx, _ = run(hsf, wls, 2, True)
    assert len(ctx.read_step_log()) == 4
    good = ctx.get_densities()
    bad = good.copy()
    bad[ctx.field_offset(1) + 5] = np.nan
    ctx.set_densities(bad)
    with pytest.raises(hsf.HsfError) as ei:
        ctx.step(1, tol=1e-9, max_iter=2000)
    assert ei.value.code == hsf.HSF_ENONFINITE
    assert ctx.read_step_log() == []
    ctx.set_densities(good)
    ctx.step(1, tol=1e-9, max_iter=2000)
    assert [r["step"] for r in ctx.read_step_log()] == [3, 3]
    ctx.step(1, tol=1e-9, max_iter=2000)
    ctx.set_step_log(False)
    assert ctx.read_step_log() == []
    ctx.step(1, tol=1e-9, max_iter=2000)
    assert ctx.read_step_log() == []
    ctx.close()


def test_step_log_counts_both_refinement_phases(hsf):
    """With FP64 refinement on (FP32 contexts), a record's counts are the step's whole
    inversion, both phases, as hsf_step's statistics give them."""
    wls = [w.with_(precision="fp32") for w in batch(True)]
    ctx = hsf.Context(wls)
    ctx.set_densities(np.concatenate([W.initial_composition(w).ravel() for w in wls]))
    ctx.set_solver(refine=True)
    ctx.set_step_log(True)
    for _ in range(2):
        stats, _ = ctx.step(1, tol=1e-9, max_iter=2000)
    recs = ctx.read_step_log()
    assert len(recs) == 4
    for r in range(2):
        rec = recs[2 + r]
        assert rec["iterations"] == stats[r]["iterations"] and rec["evaluations"] == stats[r]["evaluations"]
        assert rec["residual"] == stats[r]["residual"] and rec["residual"] <= 1e-9
    say(f"[step log, refined] {recs[-1]}")
    ctx.close()
