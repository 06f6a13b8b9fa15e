"""GPU parity: the HIP library, called through the C ABI, against the FP64 oracle
on the same seeded inputs.

Tolerances: FP64 path 1e-10 relative, FP32-propagator path 1e-5 relative
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


def osys(orc, wl, hydro=None):
    return orc.System(L=wl.L, types=wl.types, has_solvent=wl.has_solvent, a=wl.a, chi=wl.chi,
                      kappa=wl.kappa, dt=wl.dt, tau=wl.tau,
                      hydro=wl.hydro if hydro is None else hydro)


def relerr(a, b):
    """max |a - b| / max |b| over each leading-axis slice, then the max."""
    a = np.asarray(a).reshape(b.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return max(np.max(np.abs(a[i] - b[i])) / np.max(np.abs(b[i])) for i in range(b.shape[0]))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_melt(L=(16, 16, 16), types=None, precision="fp64", chiN=20.0, noise=0.01, seed=0):
    types = types or W.chain(4, 4)
    return W.Workload("test", L, types, False, W.chi_matrix(ab=chiN / len(types)), tau=1.0, noise=noise,
                      seed=seed, precision=precision)


def small_solution(L=(12, 10, 14), precision="fp64", seed=3):
    return W.Workload("test_sol", L, W.chain(3, 9), True, W.chi_matrix(ab=25 / 12, bs=35 / 12), tau=0.8,
                      noise=0.005, seed=seed, phi_p=0.12, precision=precision)


def fields_for(wl, seed, amp=1.0):
    w = W.random_fields((wl.nsp,) + wl.shape, seed=seed, amplitude=amp, smooth=1)
    return np.ascontiguousarray(w)


CASES = [
    ("melt16_a4b4", lambda p: small_melt(precision=p)),
    ("ragged17x18x20_a3b5", lambda p: small_melt(L=(17, 18, 20), types=W.chain(3, 5), precision=p)),
    ("thin33x1x5_a2b6", lambda p: small_melt(L=(33, 1, 5), types=W.chain(2, 6), precision=p)),
    ("solution12x10x14_a3b9s", lambda p: small_solution(precision=p)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_evaluate_parity(hsf, orc, name, make, precision):
    wl = make(precision)
    say(f"[evaluate] {name} {precision}")
    phi0 = W.initial_composition(wl)
    w = fields_for(wl, seed=5, amp=1.5)
    ctx = hsf.Context(wl)
    ctx.set_densities(phi0.ravel())
    ctx.set_fields(w.ravel())
    got, q = ctx.evaluate()
    pbar_p = phi0[:2].sum(0).mean()
    pbar_s = phi0[2].mean() if wl.has_solvent else 0.0
    ref, qref = orc.evaluate(osys(orc, wl), w, pbar_p, pbar_s)
    tol = TOL64 if precision == "fp64" else TOL32
    e = relerr(got, ref)
    say(f"  rel err phi {e:.3e}  Q {q[0]:.12e} vs {qref:.12e}")
    assert e < tol
    assert abs(q[0] / qref - 1) < tol
    ctx.close()


def test_homogeneous_closed_form_gpu(hsf):
    wl = small_melt(L=(8, 9, 10), types=W.chain(3, 5))
    w = np.empty((2,) + wl.shape)
    w[0], w[1] = 0.4, -0.9
    phi = np.empty_like(w)
    phi[0], phi[1] = 3 / 8, 5 / 8
    ctx = hsf.Context(wl)
    ctx.set_densities(phi.ravel())
    ctx.set_fields(w.ravel())
    got, q = ctx.evaluate()
    got = got.reshape(w.shape)
    assert abs(q[0] / np.exp(-(3 * 0.4 - 5 * 0.9)) - 1) < 1e-14
    assert np.max(np.abs(got[0] - 3 / 8)) < 1e-14 and np.max(np.abs(got[1] - 5 / 8)) < 1e-14


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fp32_scales_extreme_fields(hsf, orc, precision):
    """Strong fields whose raw propagator products leave the FP32 range: the
    per-step power-of-two scales keep the densities right (second call uses
    the scales adapted by the first)."""
    wl = small_melt(L=(12, 12, 12), types=W.chain(8, 8), precision=precision)
    phi0 = W.initial_composition(wl)
    w = fields_for(wl, seed=2, amp=1.0) - 7.0  # exp(-w) ~ e^7 per bead: G_16 ~ e^112
    ctx = hsf.Context(wl)
    ctx.set_densities(phi0.ravel())
    ctx.set_fields(w.ravel())
    ref, qref = orc.evaluate(osys(orc, wl), w, 1.0, 0.0)
    for k in range(2):
        got, q = ctx.evaluate()
        say(f"[extreme] {precision} call {k}: rel err {relerr(got, ref):.3e}, Q {q[0]:.6e} vs {qref:.6e}")
    tol = TOL64 if precision == "fp64" else TOL32
    assert relerr(got, ref) < tol
    assert abs(q[0] / qref - 1) < tol


def test_invert_parity_fp64(hsf, orc):
    wl = small_melt(L=(16, 12, 10), types=W.chain(4, 4))
    say("[invert fp64]")
    wt = fields_for(wl, seed=7, amp=0.8)
    wt -= wt.mean(axis=(1, 2, 3), keepdims=True)
    sysw = osys(orc, wl)
    phit, _ = orc.evaluate(sysw, wt, 1.0, 0.0)
    w0 = -np.log(phit / phit.mean(axis=(1, 2, 3), keepdims=True))
    _, st_tol, _ = orc.invert(sysw, phit, w0, tol=1e-10, max_iter=500)
    ctx = hsf.Context(wl)
    ctx.set_densities(phit.ravel())
    st, rcg = ctx.invert(tol=1e-10, max_iter=500, warm=hsf.WARM_LOCAL)
    # mirror mode: the oracle takes exactly the GPU's number of iterations (a stopping
    # test within rounding of the tolerance may otherwise end one iteration apart)
    wref, st_ref, rc = orc.invert(sysw, phit, w0, tol=1e-10, max_iter=500, fixed_iters=st[0]["iterations"])
    say(f"  gpu {st[0]}  oracle(tol) {st_tol}  oracle(mirror) {st_ref}")
    w = ctx.get_fields().reshape(wt.shape)
    assert st[0]["converged"] and st[0]["residual"] <= 1e-10
    assert abs(st[0]["iterations"] - st_tol["iterations"]) <= 2
    assert st[0]["evaluations"] == st_ref["evaluations"]
    # after ~100 iterations the trajectories agree to ~1e-11: compare residuals absolutely
    assert abs(st_ref["residual"] - st[0]["residual"]) < 1e-10
    assert np.max(np.abs(w - wref)) < 1e-9
    # the GPU densities at its own fields reproduce the target
    got, _ = ctx.evaluate()
    assert relerr(got, phit) < 1e-9


def test_invert_solution_fp32(hsf, orc):
    wl = small_solution(precision="fp32")
    say("[invert fp32 solution]")
    phit = W.initial_composition(wl)
    ctx = hsf.Context(wl)
    ctx.set_densities(phit.ravel())
    st, _ = ctx.invert(tol=1e-6, max_iter=500, warm=hsf.WARM_LOCAL)
    say(f"  gpu {st[0]}")
    assert st[0]["converged"]
    w = ctx.get_fields().reshape((3,) + wl.shape)
    # the FP64 oracle's densities at the GPU's fields reproduce the target: the
    # residual (relative L2 norm per polymer species) is within the tolerance
    # plus the FP32 evaluation error (about 4e-7 relative after 12 FP32 steps)
    ref, _ = orc.evaluate(osys(orc, wl), w, phit[:2].sum(0).mean(), phit[2].mean())
    res = max(np.linalg.norm(ref[I] - phit[I]) / np.linalg.norm(phit[I]) for I in range(2))
    say(f"  FP64 residual at the GPU fields {res:.3e}")
    assert res < 1e-6 + 5e-7
    assert np.max(np.abs(ref[2] - phit[2])) < 1e-14


def test_mu_force_parity(hsf, orc):
    wl = small_solution(L=(9, 11, 7))
    phi = W.initial_composition(wl)
    w = fields_for(wl, seed=4)
    ctx = hsf.Context(wl)
    ctx.set_densities(phi.ravel())
    ctx.set_fields(w.ravel())
    mu, f = ctx.mu_force()
    mref, fref = orc.mu_force(osys(orc, wl), phi, w)
    assert relerr(mu, mref) < 1e-13
    assert np.max(np.abs(f.reshape(fref.shape) - fref)) <= 1e-13 * np.max(np.abs(fref))


@pytest.mark.parametrize("L,tau", [((16, 16, 16), 0.6), ((17, 5, 9), 1.5)])
def test_lb_parity(hsf, orc, L, tau):
    wl = small_melt(L=L).with_(tau=tau)
    sysw = osys(orc, wl)
    rng = np.random.default_rng(1)
    n = orc.lb_rest_state(sysw) * (1 + 0.02 * rng.uniform(-1, 1, size=(19,) + wl.shape))
    n = np.ascontiguousarray(n)
    f = np.ascontiguousarray(1e-3 * rng.uniform(-1, 1, size=(3,) + wl.shape))
    ctx = hsf.Context(wl)
    ctx.set_lb(n.ravel())
    ctx.lb_advance(3, f.ravel())
    got = ctx.get_lb().reshape(n.shape)
    rho, u = ctx.get_flow()
    ref = n
    for _ in range(3):
        ref, rref, uref = orc.lb_step(sysw, ref, f)
    assert np.max(np.abs(got - ref)) < 1e-14
    assert np.max(np.abs(rho.reshape(rref.shape) - rref)) < 1e-14
    assert np.max(np.abs(u.reshape(uref.shape) - uref)) < 1e-15
    assert abs(got.sum() / n.sum() - 1) < 1e-14


@pytest.mark.parametrize("lb", ["bgk", "mrt"])
def test_lb_parity_fp32_storage(hsf, orc, lb):
    """FP32 contexts store the populations as FP32 deviations from the rest state (FP64
    arithmetic): three forced steps (BGK tau 0.6, or MRT with independent eigenvalues)
    against the FP64 oracle on a ragged box; the storage rounding of the deviations
    (about 2^-24 of a 2 % perturbation) stays below 1e-9 absolute, far inside 1e-5, and
    the total mass is kept to 1e-10 (each stored deviation is rounded once per step, by at
    most 2^-24 of |n_i - w_i| <= 0.02 w_i; measured 1.6e-12 over 3 steps of 765 sites)."""
    gammas = (0.3, -0.2, 0.1)
    wl = small_melt(L=(17, 5, 9), precision="fp32").with_(tau=0.6)
    if lb == "mrt":
        wl = wl.with_(lb="mrt", gammas=gammas)
    sysw = osys(orc, wl)
    if lb == "mrt":
        sysw.lb_mode = 1
        sysw.gamma_s, sysw.gamma_b, sysw.gamma_ghost = gammas
    rng = np.random.default_rng(7)
    n = np.ascontiguousarray(orc.lb_rest_state(sysw) * (1 + 0.02 * rng.uniform(-1, 1, size=(19,) + wl.shape)))
    f = np.ascontiguousarray(1e-3 * rng.uniform(-1, 1, size=(3,) + wl.shape))
    ctx = hsf.Context(wl)
    ctx.set_lb(n.ravel())
    n_in = ctx.get_lb().reshape(n.shape)   # the stored (rounded) starting populations
    assert np.max(np.abs(n_in - n)) < 1e-9
    ctx.lb_advance(3, f.ravel())
    got = ctx.get_lb().reshape(n.shape)
    rho, u = ctx.get_flow()
    ref = n_in
    for _ in range(3):
        ref, rref, uref = orc.lb_step(sysw, ref, f)
    e = np.max(np.abs(got - ref))
    say(f"[lb fp32 {lb}] max |dn| {e:.2e}")
    assert e < 1e-9
    assert np.max(np.abs(rho.reshape(rref.shape) - rref)) < 1e-9
    assert np.max(np.abs(u.reshape(uref.shape) - uref)) < 1e-9
    assert abs(got.sum() / n_in.sum() - 1) < 1e-10


@pytest.mark.parametrize("gammas", [(0.3, -0.2, 0.1), (-0.5, 0.4, -0.3), (0.0, 0.0, 0.0)])
def test_lb_mrt_parity(hsf, orc, gammas):
    """The multiple-relaxation-time collision of eq. 12-14 in the basis of Table 1,
    with independent shear, bulk and kinetic-mode eigenvalues, against the oracle's."""
    wl = small_melt(L=(9, 7, 11)).with_(lb="mrt", gammas=gammas)
    sysw = osys(orc, wl)
    sysw.lb_mode = 1
    sysw.gamma_s, sysw.gamma_b, sysw.gamma_ghost = gammas
    rng = np.random.default_rng(4)
    n = orc.lb_rest_state(sysw) * (1 + 0.03 * rng.uniform(-1, 1, size=(19,) + wl.shape))
    n = np.ascontiguousarray(n)
    f = np.ascontiguousarray(2e-3 * rng.uniform(-1, 1, size=(3,) + wl.shape))
    ctx = hsf.Context(wl)
    ctx.set_lb(n.ravel())
    ctx.lb_advance(3, f.ravel())
    got = ctx.get_lb().reshape(n.shape)
    rho, u = ctx.get_flow()
    ref = n
    for _ in range(3):
        ref, rref, uref = orc.lb_step(sysw, ref, f)
    e = np.max(np.abs(got - ref))
    say(f"[lb mrt {gammas}] max |dn| {e:.2e}")
    assert e < 1e-14
    assert np.max(np.abs(rho.reshape(rref.shape) - rref)) < 1e-14
    assert np.max(np.abs(u.reshape(uref.shape) - uref)) < 1e-15
    assert abs(got.sum() / n.sum() - 1) < 1e-14


def test_mrt_trajectory_fp64(hsf, orc):
    """Ten coupled steps of the 16^3 A4B4 melt with the MRT collision (shear viscosity of
    tau = 0.8, bulk eigenvalue of tau 1.2, kinetic modes relaxed completely), GPU
    against the oracle in mirror mode."""
    g = W.mrt_gammas(0.8, 1.2, 0.0)
    wl = W.melt16_a4b4().with_(lb="mrt", gammas=g)
    sysw = osys(orc, wl)
    sysw.lb_mode = 1
    sysw.gamma_s, sysw.gamma_b, sysw.gamma_ghost = g
    phi = W.initial_composition(wl)
    ctx = hsf.Context(wl)
    ctx.set_densities(phi.ravel())
    w = -np.log(phi / phi.mean(axis=(1, 2, 3), keepdims=True))
    ctx.set_fields(w.ravel())
    n = orc.lb_rest_state(sysw)
    for k in range(10):
        st, _ = ctx.step(1, tol=wl.tol, max_iter=1000)
        phi, w, n, st_ref, u, rho, rc = orc.step(sysw, phi, w, n, tol=wl.tol, max_iter=1000,
                                                 fixed_iters=st[0]["iterations"])
        got = ctx.get_densities().reshape(phi.shape)
        assert relerr(got, phi) < TOL64, k
    ng = ctx.get_lb().reshape(n.shape)
    assert np.max(np.abs(ng - n)) < 1e-13
    say(f"[mrt trajectory] max |dn| after 10 steps {np.max(np.abs(ng - n)):.2e}")


def test_cd_parity(hsf, orc):
    wl = small_solution(L=(10, 7, 12))
    rng = np.random.default_rng(2)
    phi = W.initial_composition(wl)
    mu = rng.standard_normal((3,) + wl.shape)
    u = 0.05 * rng.standard_normal((3,) + wl.shape)
    ctx = hsf.Context(wl)
    ctx.set_densities(phi.ravel())
    ctx.cd_advance(mu.ravel(), u.ravel())
    got = ctx.get_densities().reshape(phi.shape)
    ref = orc.cd_update(osys(orc, wl), phi, mu, u)
    assert np.max(np.abs(got - ref)) < 1e-15
    assert np.max(np.abs(got.sum(axis=(1, 2, 3)) / phi.sum(axis=(1, 2, 3)) - 1)) < 1e-13


def test_melt16_trajectory_fp64(hsf, orc):
    """16^3 A4B4 melt, chi N = 20, tau 1.0, residual 1e-8: 100 coupled steps,
    GPU against the oracle, step by step."""
    wl = W.melt16_a4b4()
    say("[trajectory melt16_a4b4 fp64 100 steps]")
    phi = W.initial_composition(wl)
    sysw = osys(orc, wl)
    ctx = hsf.Context(wl)
    ctx.set_densities(phi.ravel())
    w = -np.log(phi / phi.mean(axis=(1, 2, 3), keepdims=True))
    ctx.set_fields(w.ravel())
    n = orc.lb_rest_state(sysw)
    worst = 0.0
    for k in range(wl.steps):
        st, _ = ctx.step(1, tol=wl.tol, max_iter=1000)
        # mirror mode: the oracle's inversion takes the GPU's iteration count of this step
        phi, w, n, st_ref, u, rho, rc = orc.step(sysw, phi, w, n, tol=wl.tol, max_iter=1000,
                                                 fixed_iters=st[0]["iterations"])
        got = ctx.get_densities().reshape(phi.shape)
        e = relerr(got, phi)
        worst = max(worst, e)
        if k % 20 == 0 or e > TOL64:
            say(f"  step {k}: iters {st[0]['iterations']} residual gpu {st[0]['residual']:.3e} "
                f"oracle {st_ref['residual']:.3e}  rel err {e:.3e}")
        assert st[0]["converged"] and st_ref["residual"] <= 1.01 * wl.tol, (k, st[0], st_ref)
        assert e < TOL64, k
    wg = ctx.get_fields().reshape(w.shape)
    assert np.max(np.abs(wg - w)) < 1e-8
    ng = ctx.get_lb().reshape(n.shape)
    assert np.max(np.abs(ng - n)) < 1e-14
    say(f"  worst rel err over 100 steps {worst:.3e}")


def test_batched_replicas_match_single(hsf, orc):
    """Uneven boxes in one context: each replica equals the oracle."""
    wls = [small_solution(L=(8, 8, 8), seed=1, precision="fp64"),
           small_solution(L=(12, 10, 6), seed=2, precision="fp64").with_(chi=W.chi_matrix(ab=1.9, bs=2.5)),
           small_solution(L=(5, 9, 11), seed=3, precision="fp64").with_(chi=W.chi_matrix(ab=2.6, bs=2.2))]
    ctx = hsf.Context(wls)
    phis = [W.initial_composition(wl) for wl in wls]
    ctx.set_densities(np.concatenate([p.ravel() for p in phis]))
    ctx.set_fields(np.concatenate([(-np.log(p / p.mean(axis=(1, 2, 3), keepdims=True))).ravel() for p in phis]))
    st, _ = ctx.step(3, tol=1e-9, max_iter=1000)
    got = ctx.get_densities()
    for r, wl in enumerate(wls):
        sysw = osys(orc, wl)
        phi = phis[r]
        w = -np.log(phi / phi.mean(axis=(1, 2, 3), keepdims=True))
        n = orc.lb_rest_state(sysw)
        for _ in range(3):
            phi, w, n, st_ref, _, _, _ = orc.step(sysw, phi, w, n, tol=1e-9, max_iter=1000)
        o = ctx.field_offset(r)
        g = got[o:o + phi.size].reshape(phi.shape)
        e = relerr(g, phi)
        say(f"[batch] replica {r} {wl.L}: rel err {e:.3e}, iters {st[r]['iterations']} vs {st_ref['iterations']}")
        assert e < TOL64


def test_full_size_melt64_fp32_sampled(hsf, orc):
    """64^3 A8B8 melt with FP32 propagators, the bench's launch configuration:
    one evaluation compared with the oracle at every site (the oracle runs the
    full box in about a second), plus the FP64 path."""
    for precision, tol in (("fp32", TOL32), ("fp64", TOL64)):
        wl = W.melt64_a8b8(precision=precision)
        phi0 = W.initial_composition(wl)
        w = fields_for(wl, seed=11, amp=1.0)
        ctx = hsf.Context(wl)
        ctx.set_densities(phi0.ravel())
        ctx.set_fields(w.ravel())
        got, q = ctx.evaluate()
        ref, qref = orc.evaluate(osys(orc, wl), w, 1.0, 0.0)
        e = relerr(got, ref)
        say(f"[melt64 {precision}] rel err {e:.3e}")
        assert e < tol and abs(q[0] / qref - 1) < tol
        ctx.close()


def test_graph_replays_match_direct_launches(hsf, orc, monkeypatch):
    """The captured launch sequences, replayed many times with eager work and
    synchronisations in between, give bit-identical results to direct launches."""
    wl = small_solution(L=(10, 9, 8), precision="fp32")
    phi = W.initial_composition(wl)
    out = []
    for no_graphs in ("1", "0"):
        monkeypatch.setenv("HSF_NO_GRAPHS", no_graphs)
        ctx = hsf.Context(wl)
        ctx.set_densities(phi.ravel())
        res = []
        for k in range(4):
            st, _ = ctx.step(1, tol=1e-6)
            e, _ = ctx.evaluate()
            res.append((ctx.get_densities().copy(), ctx.get_fields().copy(), e.copy(), st[0]["evaluations"]))
        out.append(res)
        ctx.close()
    for (a, b) in zip(out[0], out[1]):
        assert a[3] == b[3]
        for x, y in zip(a[:3], b[:3]):
            assert np.array_equal(x, y)


TILES = [(64, 4, 1, 0), (32, 8, 1, 0), (16, 16, 1, 0), (64, 4, 2, 0), (32, 8, 2, 0), (16, 16, 2, 0), (64, 4, 4, 0),
         (32, 8, 4, 0), (16, 16, 4, 0), (64, 4, 8, 0), (16, 16, 8, 0), (8, 8, 8, 1), (8, 8, 8, 2), (8, 8, 8, 3), (8, 8, 8, 4), (16, 8, 8, 2), (16, 8, 4, 2), (32, 8, 4, 1),
         (32, 4, 4, 2), (64, 4, 2, -1), (64, 4, 4, -1), (32, 8, 2, -1), (16, 16, 2, -1), (32, 8, 4, -1), (16, 16, 4, -1),
         (16, 16, 8, -1), (64, 8, 8, 2), (64, 8, 16, 2), (64, 16, 8, 2), (64, 16, 16, 2), (64, 16, 32, 2)]
PAIRED = [t for t in TILES if t[3] == -1]
STREAM = [t for t in TILES if t[0] == 64 and t[3] >= 1]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_every_tile_configuration(hsf, orc, precision):
    """Every compiled tiling of the blocked sweeps gives the oracle's densities, on
    boxes that are ragged against every tile and smaller than the halo (N not a
    multiple of k either)."""
    cases = [small_melt(L=L, types=types, precision=precision) for L, types in
             [((17, 18, 20), W.chain(3, 4)), ((5, 3, 9), W.chain(2, 3)), ((40, 9, 6), W.chain(4, 4)),
              ((70, 23, 11), W.chain(1, 3))]]
    cases.append(small_solution(L=(12, 10, 14), precision=precision))
    for wl in cases:
        L = wl.L
        phi0 = W.initial_composition(wl)
        w = fields_for(wl, seed=9, amp=1.2)
        pbar = phi0[:2].sum(0).mean()
        ref, qref = orc.evaluate(osys(orc, wl), w, pbar, phi0[2].mean() if wl.has_solvent else 0.0)
        ctx = hsf.Context(wl)
        ctx.set_densities(phi0.ravel())
        ctx.set_fields(w.ravel())
        for t in TILES:
            try:
                ctx.set_tile(t)
            except hsf.HsfError:
                continue  # over the device's LDS limit
            got, q = ctx.evaluate()
            e = relerr(got, ref)
            say(f"[tile {t}] {L} {precision}: rel err {e:.3e}")
            tol = TOL64 if precision == "fp64" else TOL32
            assert e < tol and abs(q[0] / qref - 1) < tol, (t, L)
        ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_every_tile_configuration_batched(hsf, orc, precision):
    """The same with two replicas of uneven boxes in one context (the replica of each
    block comes from the tile plan, not a kernel argument)."""
    types = W.chain(3, 4)
    wls = [small_melt(L=(17, 18, 20), types=types, precision=precision, seed=1),
           small_melt(L=(5, 3, 9), types=types, precision=precision, seed=2)]
    ws = [fields_for(wl, seed=9 + r, amp=1.2) for r, wl in enumerate(wls)]
    refs = [orc.evaluate(osys(orc, wl), w, 1.0, 0.0) for wl, w in zip(wls, ws)]
    ctx = hsf.Context(wls)
    ctx.set_densities(np.concatenate([W.initial_composition(wl).ravel() for wl in wls]))
    ctx.set_fields(np.concatenate([w.ravel() for w in ws]))
    tol = TOL64 if precision == "fp64" else TOL32
    for t in TILES:
        try:
            ctx.set_tile(t)
        except hsf.HsfError:
            continue
        got, q = ctx.evaluate()
        for r, (wl, (ref, qref)) in enumerate(zip(wls, refs)):
            fo = ctx.field_offset(r)
            e = relerr(got[fo:fo + 2 * wl.V], ref)
            say(f"[tile {t} batched] replica {r} {precision}: rel err {e:.3e}")
            assert e < tol and abs(q[r] / qref - 1) < tol, (t, r)
    ctx.close()


def test_autotune_keeps_results(hsf, orc):
    wl = small_melt(L=(32, 32, 32), types=W.chain(4, 4), precision="fp32")
    phi0 = W.initial_composition(wl)
    w = fields_for(wl, seed=3)
    ctx = hsf.Context(wl)
    ctx.set_densities(phi0.ravel())
    ctx.set_fields(w.ravel())
    cfg, ms = ctx.autotune(reps=2)
    say(f"[autotune] chose {cfg} at {ms:.3f} ms per evaluation")
    assert tuple(cfg) in [tuple(t) for t in TILES]
    assert np.array_equal(ctx.get_fields(), w.ravel())
    got, q = ctx.evaluate()
    ref, qref = orc.evaluate(osys(orc, wl), w, 1.0, 0.0)
    assert relerr(got, ref) < TOL32


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_preconditioned_inversion(hsf, orc, precision):
    """Diagonally preconditioned variant: GPU against the oracle's same variant in
    mirror mode; it reaches the same residual in fewer evaluations on a solution."""
    wl = small_solution(L=(12, 12, 12), precision=precision)
    phit = W.initial_composition(wl)
    sysw = osys(orc, wl)
    sysw.precond = True
    ctx = hsf.Context(wl)
    ctx.set_solver(precond=True)
    ctx.set_densities(phit.ravel())
    tol = 1e-9 if precision == "fp64" else 1e-6
    st, _ = ctx.invert(tol=tol, max_iter=2000, warm=hsf.WARM_LOCAL)
    w0 = -np.log(phit / phit.mean(axis=(1, 2, 3), keepdims=True))
    wref, st_ref, _ = orc.invert(sysw, phit, w0, tol=tol, max_iter=2000, fixed_iters=st[0]["iterations"])
    sysw.precond = False
    _, st_plain, _ = orc.invert(sysw, phit, w0, tol=tol, max_iter=2000)
    say(f"[precond {precision}] gpu {st[0]} oracle(mirror) {st_ref} oracle plain FR {st_plain}")
    assert st[0]["converged"]
    assert st[0]["evaluations"] < st_plain["evaluations"]
    w = ctx.get_fields().reshape(wref.shape)
    wg = w - w.mean(axis=(1, 2, 3), keepdims=True)
    wr = wref - wref.mean(axis=(1, 2, 3), keepdims=True)
    if precision == "fp64":
        assert st[0]["evaluations"] == st_ref["evaluations"]
        assert np.max(np.abs(wg - wr)) < 1e-8
    else:
        assert np.max(np.abs(wg - wr)) < 1e-3


@pytest.mark.parametrize("n_rep", [4, 5])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_kernel_modes(hsf, orc, n_rep, precision):
    """Batches of up to four replicas pass their descriptors to the propagator kernels as
    arguments, larger ones read them from device tables: uneven boxes at the boundary of
    the two (4 and 5 replicas), one replica made inactive by converging first, evaluated
    and inverted in the one-step and in a blocked tiling; every replica matches the oracle."""
    boxes = [(8, 8, 8), (12, 10, 6), (5, 9, 11), (7, 6, 9), (10, 5, 8)][:n_rep]
    wls = [small_solution(L=L, seed=10 + k, precision=precision) for k, L in enumerate(boxes)]
    say(f"[batch modes] {n_rep} replicas {precision}")
    phis = [W.initial_composition(wl) for wl in wls]
    ws = [fields_for(wl, seed=40 + k, amp=0.8) for k, wl in enumerate(wls)]
    tol = TOL64 if precision == "fp64" else TOL32
    for tile in ((64, 4, 2, 0), (8, 8, 8, 2)):
        ctx = hsf.Context(wls)
        ctx.set_tile(tile)
        ctx.set_densities(np.concatenate([p.ravel() for p in phis]))
        ctx.set_fields(np.concatenate([w.ravel() for w in ws]))
        got, q = ctx.evaluate()
        for r, wl in enumerate(wls):
            o = ctx.field_offset(r)
            ref, qref = orc.evaluate(osys(orc, wl), ws[r], phis[r][:2].sum(0).mean(), phis[r][2].mean())
            e = relerr(got[o:o + ref.size].reshape(ref.shape), ref)
            assert e < tol and abs(q[r] / qref - 1) < tol, (tile, r, e)
        # an inversion in which the replicas finish at different iterations: the densities
        # at each replica's final fields reproduce its target
        st, _ = ctx.invert(tol=1e-8 if precision == "fp64" else 1e-6, max_iter=2000, warm=hsf.WARM_LOCAL)
        its = [s["iterations"] for s in st]
        assert all(s["converged"] for s in st) and len(set(its)) > 1, its
        wf = ctx.get_fields()
        for r, wl in enumerate(wls):
            o = ctx.field_offset(r)
            w = wf[o:o + phis[r].size].reshape(phis[r].shape)
            ref, _ = orc.evaluate(osys(orc, wl), w, phis[r][:2].sum(0).mean(), phis[r][2].mean())
            res = max(np.linalg.norm(ref[I] - phis[r][I]) / np.linalg.norm(phis[r][I]) for I in range(2))
            assert res < (1e-8 if precision == "fp64" else 1e-6 + 5e-7), (tile, r, res)
        say(f"  tile {tile}: evaluate ok, inversion iterations {its}")
        ctx.close()


@pytest.mark.parametrize("types,L", [([0], (9, 7, 5)), ([1], (6, 8, 5)), (W.chain(1, 1), (7, 6, 9)),
                                     (W.chain(32, 32), (10, 9, 8)), (W.chain(5, 59), (6, 6, 7))],
                         ids=["n1_a", "n1_b", "n2_a1b1", "n64_a32b32", "n64_a5b59"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_chain_length_extremes(hsf, orc, types, L, precision):
    """Single-bead chains (step 1 is step N: Q cannot be folded into the first backward
    step), the shortest diblock and the longest chain the library takes (64 beads: every
    slot of the per-step scales and the stored propagators in use), in a one-step and a
    blocked tiling.  A species the chain does not contain has density exactly zero."""
    wl = small_melt(L=L, types=types, precision=precision)
    N = len(types)
    frac = np.array([types.count(0) / N, types.count(1) / N])
    phi0 = np.ascontiguousarray(np.broadcast_to(frac[:, None, None, None], (2,) + wl.shape))
    w = fields_for(wl, seed=13, amp=1.5)
    ref, qref = orc.evaluate(osys(orc, wl), w, 1.0, 0.0)
    tol = TOL64 if precision == "fp64" else TOL32
    ctx = hsf.Context(wl)
    ctx.set_densities(phi0.ravel())
    ctx.set_fields(w.ravel())
    for tile in ((64, 4, 2, 0), (8, 8, 8, 2), (64, 4, 2, -1)):
        ctx.set_tile(tile)
        got, q = ctx.evaluate()
        got = got.reshape(ref.shape)
        errs = []
        for i in range(2):
            if frac[i] == 0:
                assert np.all(got[i] == 0.0), (tile, i)
            else:
                errs.append(np.max(np.abs(got[i] - ref[i])) / np.max(np.abs(ref[i])))
        say(f"[chain N={N} {types[:3]}...] {precision} tile {tile}: rel err {max(errs):.3e}, "
            f"Q {q[0]:.6e} vs {qref:.6e}")
        assert max(errs) < tol and abs(q[0] / qref - 1) < tol, tile
    ctx.close()


@pytest.mark.parametrize("L", [(1, 1, 1), (2, 1, 1), (1, 3, 1), (1, 1, 2)], ids=lambda L: "x".join(map(str, L)))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_smallest_boxes(hsf, orc, L, precision):
    """Boxes of one to three sites, where every neighbour of the 27-point stencil wraps
    onto the same few sites: densities and Q against the oracle in a one-step and a
    blocked tiling, then one coupled step (inversion, LB, convection-diffusion) keeps
    each species' amount and stays finite."""
    wl = small_melt(L=L, types=W.chain(2, 3), precision=precision)
    phi0 = W.initial_composition(wl)
    w = fields_for(wl, seed=17, amp=1.0)
    ref, qref = orc.evaluate(osys(orc, wl), w, phi0.sum(0).mean(), 0.0)
    tol = TOL64 if precision == "fp64" else TOL32
    ctx = hsf.Context(wl)
    ctx.set_densities(phi0.ravel())
    ctx.set_fields(w.ravel())
    for tile in ((64, 4, 2, 0), (8, 8, 8, 2), (32, 8, 2, -1)):
        ctx.set_tile(tile)
        got, q = ctx.evaluate()
        e = relerr(got, ref)
        say(f"[box {L}] {precision} tile {tile}: rel err {e:.3e}, Q {q[0]:.6e} vs {qref:.6e}")
        assert e < tol and abs(q[0] / qref - 1) < tol, tile
    st, _ = ctx.step(1, tol=1e-10 if precision == "fp64" else 1e-6, max_iter=500)
    assert st[0]["converged"]
    phi1 = ctx.get_densities().reshape(phi0.shape)
    assert np.all(np.isfinite(phi1))
    assert np.max(np.abs(phi1.sum(axis=(1, 2, 3)) - phi0.sum(axis=(1, 2, 3)))) < 1e-12
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_error_paths_and_recovery(hsf, orc, precision):
    """The boundary's error returns on the GPU path, and that a context is usable after
    each: an inversion stopped at max_iter returns HSF_ENOCONV and keeps its iterate, from
    which a second inversion converges; a non-finite field makes the evaluation return
    HSF_ENONFINITE, and after finite fields are set again the context evaluates bit for
    bit as before; bad arguments return HSF_EINVAL and change nothing."""
    wl = small_melt(L=(12, 10, 9), types=W.chain(3, 5), precision=precision)
    tol = 1e-10 if precision == "fp64" else 1e-6
    phi0 = W.initial_composition(wl)
    ctx = hsf.Context(wl)
    ctx.set_densities(phi0.ravel())
    # HSF_ENOCONV, then convergence from the kept iterate
    st, rc = ctx.invert(tol=tol, max_iter=2, warm=hsf.WARM_LOCAL, allow_noconv=True)
    assert rc == hsf.HSF_ENOCONV and st[0]["iterations"] == 2 and not st[0]["converged"]
    with pytest.raises(hsf.HsfError) as ei:
        ctx.invert(tol=tol, max_iter=1, warm=hsf.WARM_CURRENT)
    assert ei.value.code == hsf.HSF_ENOCONV
    w_kept = ctx.get_fields()
    assert np.all(np.isfinite(w_kept))
    st, rc = ctx.invert(tol=tol, max_iter=2000, warm=hsf.WARM_CURRENT)
    assert rc == hsf.HSF_OK and st[0]["converged"] and st[0]["residual"] <= tol
    # HSF_ENONFINITE and recovery
    w_good = ctx.get_fields()
    ref, q_ref = ctx.evaluate()
    w_bad = w_good.copy()
    w_bad[wl.V // 2] = np.nan
    ctx.set_fields(w_bad)
    with pytest.raises(hsf.HsfError) as ei:
        ctx.evaluate()
    assert ei.value.code == hsf.HSF_ENONFINITE
    ctx.set_fields(w_good)
    got, q = ctx.evaluate()
    assert np.array_equal(got, ref) and np.array_equal(q, q_ref)
    # HSF_EINVAL leaves the state alone
    for call in (lambda: ctx.invert(tol=-1.0), lambda: ctx.invert(tol=tol, max_iter=-1),
                 lambda: ctx.invert(tol=tol, warm=99), lambda: ctx.set_tile((3, 3, 3, 0)),
                 lambda: ctx.step(-1)):
        with pytest.raises(hsf.HsfError) as ei:
            call()
        assert ei.value.code == hsf.HSF_EINVAL
    assert np.array_equal(ctx.get_fields(), w_good)
    got, q = ctx.evaluate()
    assert np.array_equal(got, ref) and np.array_equal(q, q_ref)
    ctx.close()


def test_user_stream_and_device_buffers(hsf):
    """A context on a caller's stream (a torch stream other than the default), fed with
    device tensors written on that stream and evaluating into a device tensor, gives bit
    for bit the densities, Q and 3-step trajectory of a context on the default stream fed
    from host arrays."""
    import torch
    wl = small_melt(L=(12, 10, 9), types=W.chain(3, 5), precision="fp32")
    phi0 = W.initial_composition(wl)
    w = fields_for(wl, seed=3, amp=1.0)
    ref = hsf.Context(wl)
    ref.set_densities(phi0.ravel())
    ref.set_fields(w.ravel())
    r_phi, r_q = ref.evaluate()
    ref.step(3, tol=1e-6, max_iter=500)
    r_after, r_w = ref.get_densities(), ref.get_fields()
    ref.close()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        phi_d = torch.from_numpy(phi0.ravel().copy()).to("cuda")
        w_d = torch.from_numpy(w.ravel().copy()).to("cuda")
        out = torch.full_like(phi_d, float("nan"))
    ctx = hsf.Context(wl, stream=s)
    ctx.set_densities(phi_d)
    ctx.set_fields(w_d)
    _, q = ctx.evaluate(out=out)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), r_phi) and np.array_equal(q, r_q)
    ctx.step(3, tol=1e-6, max_iter=500)
    assert np.array_equal(ctx.get_densities(), r_after) and np.array_equal(ctx.get_fields(), r_w)
    ctx.close()


def test_hydro_switched_mid_run(hsf, orc):
    """Convection switched off and on again during a run (16^3 A4B4, FP64, residual 1e-8):
    three coupled steps with the LB flow, three purely diffusive (the LB state kept), three
    with the flow again, GPU against the oracle step by step in mirror mode; the LB
    populations at the end agree too."""
    wl = W.melt16_a4b4()
    phi = W.initial_composition(wl)
    sysw = osys(orc, wl)
    ctx = hsf.Context(wl)
    ctx.set_densities(phi.ravel())
    w = -np.log(phi / phi.mean(axis=(1, 2, 3), keepdims=True))
    ctx.set_fields(w.ravel())
    n = orc.lb_rest_state(sysw)
    for k, hydro in enumerate([True] * 3 + [False] * 3 + [True] * 3):
        ctx.set_hydro(hydro)
        sysw.hydro = hydro
        st, _ = ctx.step(1, tol=wl.tol, max_iter=1000)
        phi, w, n, st_ref, _, _, _ = orc.step(sysw, phi, w, n, tol=wl.tol, max_iter=1000,
                                               fixed_iters=st[0]["iterations"])
        e = relerr(ctx.get_densities().reshape(phi.shape), phi)
        say(f"[hydro switch] step {k} hydro {hydro}: rel err {e:.3e}")
        assert st[0]["converged"] and e < TOL64, k
        if k == 5:   # the populations did not move while the flow was off
            assert np.max(np.abs(ctx.get_lb().reshape(n.shape) - n)) < 1e-14
    assert np.max(np.abs(ctx.get_lb().reshape(n.shape) - n)) < 1e-14
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_paired_sweeps_match_one_step_bitwise(hsf, orc, precision):
    """Paired launches (one forward and one backward contour step per launch, the
    density term formed by whichever of a bead's two steps runs second) store every
    value as the same expression of the same operands as the one-step sequence: for
    odd and even N (N = 2, where backward step N forms its own field factor, and even
    N >= 4, where backward step N - 1 forms G+_N from the stored factor), one replica
    (descriptors as kernel arguments) and six of uneven
    boxes (descriptors in device tables), the densities and Q are bit for bit those of
    the one-step kernels of the same tiling, and within tolerance of the oracle."""
    tol = TOL64 if precision == "fp64" else TOL32
    for L, types in [((17, 18, 20), W.chain(3, 4)), ((24, 20, 9), W.chain(4, 4)), ((5, 3, 9), W.chain(2, 3)),
                     ((9, 7, 5), W.chain(1, 1)), ((12, 11, 10), W.chain(5, 11)), ((13, 9, 11), W.chain(1, 3))]:
        wl = small_melt(L=L, types=types, precision=precision)
        w = fields_for(wl, seed=21, amp=1.2)
        ref, qref = orc.evaluate(osys(orc, wl), w, 1.0, 0.0)
        ctx = hsf.Context(wl)
        ctx.set_densities(W.initial_composition(wl).ravel())
        ctx.set_fields(w.ravel())
        for t in PAIRED:
            ctx.set_tile(t[:3] + (0,))
            ctx.evaluate()   # the FP32 scales follow the previous evaluation: same state for both
            one, q1 = ctx.evaluate()
            ctx.set_tile(t)
            two, q2 = ctx.evaluate()
            say(f"[paired {t}] {L} N={len(types)} {precision}: rel err {relerr(two, ref):.3e}")
            assert np.array_equal(one, two) and np.array_equal(q1, q2), (t, L)
            assert relerr(two, ref) < tol and abs(q2[0] / qref - 1) < tol, (t, L)
        ctx.close()
    types = W.chain(3, 4)
    wls = [small_melt(L=Lr, types=types, precision=precision, seed=r)
           for r, Lr in enumerate([(17, 18, 20), (5, 3, 9), (16, 16, 16), (9, 7, 5), (20, 6, 11), (8, 8, 8)])]
    ws = [fields_for(wl, seed=30 + r, amp=1.2) for r, wl in enumerate(wls)]
    ctx = hsf.Context(wls)
    ctx.set_densities(np.concatenate([W.initial_composition(wl).ravel() for wl in wls]))
    ctx.set_fields(np.concatenate([w.ravel() for w in ws]))
    for t in PAIRED:
        ctx.set_tile(t[:3] + (0,))
        ctx.evaluate()
        one, q1 = ctx.evaluate()
        ctx.set_tile(t)
        two, q2 = ctx.evaluate()
        assert np.array_equal(one, two) and np.array_equal(q1, q2), t
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_paired_sweeps_coupled_steps_bitwise(hsf, orc, precision):
    """Three coupled steps (inversions with their line searches, LB, convection-diffusion)
    with the paired kernels leave the same densities, fields and Q bit for bit as with the
    one-step kernels of the same tiling, for a two-replica context."""
    types = W.chain(4, 4)
    wls = [small_melt(L=(20, 18, 16), types=types, precision=precision, seed=3),
           small_melt(L=(12, 12, 12), types=types, precision=precision, seed=4)]
    out = []
    for t in [(32, 8, 2, 0), (32, 8, 2, -1)]:
        ctx = hsf.Context(wls)
        ctx.set_tile(t)
        ctx.set_densities(np.concatenate([W.initial_composition(wl).ravel() for wl in wls]))
        ctx.step(3, tol=1e-8 if precision == "fp64" else 1e-6, max_iter=1000)
        out.append((ctx.get_densities(), ctx.get_fields()))
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("kind", ["melt", "solution"])
def test_fp32_refinement_below_the_fp32_floor(hsf, orc, kind):
    """FP32 contexts with HSF_SOLVER_REFINE reach a residual the FP32 evaluations cannot
    (1e-10; on these boxes FP32 alone stalls near 3e-6): without the flag the inversion stops at
    max_iter; with it the FP64 oracle's densities at the GPU's fields reproduce the target
    to 1e-9 relative, the fields equal those of an FP64 context after gauge fixing (1e-7
    relative), and the statistics add both phases.  Coupled steps with the flag keep every
    step's residual below the tolerance; a context on a caller's tiling that does not fit
    FP64 LDS refuses the flag."""
    if kind == "melt":
        wl = small_melt(L=(16, 12, 10), types=W.chain(4, 4)).with_(precision="fp32")
        sysw = osys(orc, wl)
        wt = fields_for(wl, seed=7, amp=0.8)
        phit, _ = orc.evaluate(sysw, wt - wt.mean(axis=(1, 2, 3), keepdims=True), 1.0, 0.0)
    else:
        wl = small_solution(precision="fp32")
        sysw = osys(orc, wl)
        phit = W.initial_composition(wl)
    say(f"[refine {kind}]")
    ctx = hsf.Context(wl)
    ctx.set_densities(phit.ravel())
    st, rc = ctx.invert(tol=1e-10, max_iter=200, warm=hsf.WARM_LOCAL, allow_noconv=True)
    say(f"  fp32 alone: {st[0]}")
    assert rc == hsf.HSF_ENOCONV and st[0]["residual"] > 1e-8
    ctx.set_solver(refine=True)
    ctx.set_fields(np.zeros(ctx.nsp * ctx.T))
    st, rc = ctx.invert(tol=1e-10, max_iter=2000, warm=hsf.WARM_LOCAL)
    say(f"  refined: {st[0]}")
    assert rc == hsf.HSF_OK and st[0]["converged"] and st[0]["residual"] <= 1e-10
    w = ctx.get_fields().reshape((wl.nsp,) + wl.shape)
    phibar_s = phit[2].mean() if wl.nsp == 3 else 0.0
    ref, _ = orc.evaluate(sysw, w, phit[:2].sum(0).mean(), phibar_s)
    e = max(np.max(np.abs(ref[I] - phit[I])) / np.max(np.abs(phit[I])) for I in range(wl.nsp))
    say(f"  FP64 oracle residual at the refined fields {e:.2e}")
    assert e < 1e-9
    c64 = hsf.Context(wl.with_(precision="fp64"))
    c64.set_densities(phit.ravel())
    c64.invert(tol=1e-11, max_iter=2000, warm=hsf.WARM_LOCAL)
    w64 = c64.get_fields().reshape(w.shape)
    for I in range(2):
        d = (w[I] - w[I].mean()) - (w64[I] - w64[I].mean())
        assert np.max(np.abs(d)) <= 1e-7 * max(1.0, np.max(np.abs(w64[I]))), I
    c64.close()
    # coupled steps with refinement
    ctx.set_densities(W.initial_composition(wl).ravel())
    for _ in range(3):
        st, _ = ctx.step(1, tol=1e-9, max_iter=2000)
        assert st[0]["converged"] and st[0]["residual"] <= 1e-9
    ctx.close()


def test_refinement_refuses_tilings_that_do_not_fit(hsf):
    """The 8x8x8 tiling with 4 levels needs 40 KiB of LDS in FP32 and 72 KiB in FP64: where
    the device's limit per workgroup lies between the two, the flag is refused while that
    tiling is in use, and while the flag is on hsf_set_tile refuses that tiling."""
    wl = small_melt(L=(16, 16, 16), types=W.chain(4, 4)).with_(precision="fp32")
    ctx = hsf.Context(wl)
    ctx.set_tile((8, 8, 8, 4))
    try:
        ctx.set_solver(refine=True)
    except hsf.HsfError as e:
        assert e.code == hsf.HSF_EINVAL
        ctx.set_tile((32, 8, 2, -1))
        ctx.set_solver(refine=True)
        with pytest.raises(hsf.HsfError) as ei:
            ctx.set_tile((8, 8, 8, 4))
        assert ei.value.code == hsf.HSF_EINVAL
        ctx.set_solver(refine=False)
        ctx.set_tile((8, 8, 8, 4))
        say("[refine tiles] 8x8x8x4 refused with refinement on")
    else:
        say("[refine tiles] the LDS limit holds the FP64 8x8x8x4 tiling: nothing to refuse")
    ctx.close()
