"""GPU parity of the thermal noise (LB mode noise of eq. 13, composition noise of eq. 5)
against the FP64 oracle on the same generator counters, through the C ABI.

Both sides draw the same Philox4x64-10 words (integer arithmetic, identical); the
Box-Muller normals differ only by the last-ulp differences of log, sin and cos between
the device and host math libraries, so the tolerances are those of the noise-free
parity tests (1e-14 absolute on populations and densities after a few steps, 1e-10
relative for coupled trajectories in mirror mode).
"""
import sys

import numpy as np
import pytest

from paper_1204_2088_amd import workloads as W

pytestmark = pytest.mark.gpu

OMEGA = 400.0


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


def osys(orc, wl, **kw):
    s = orc.System(L=wl.L, types=wl.types, has_solvent=wl.has_solvent, a=wl.a, chi=wl.chi,
                   kappa=wl.kappa, dt=wl.dt, tau=wl.tau, hydro=wl.hydro)
    if wl.lb == "mrt":
        s.lb_mode = 1
        s.gamma_s, s.gamma_b, s.gamma_ghost = wl.gammas
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def relerr(a, b):
    a = np.asarray(a).reshape(b.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return max(np.max(np.abs(a[i] - b[i])) / np.max(np.abs(b[i])) for i in range(b.shape[0]))


def small_melt(L=(16, 16, 16), types=None, seed=0):
    types = types or W.chain(4, 4)
    return W.Workload("noise_melt", L, types, False, W.chi_matrix(ab=20.0 / len(types)), tau=1.0, noise=0.01,
                      seed=seed, precision="fp64")


def small_solution(L=(12, 10, 14), seed=3):
    return W.Workload("noise_sol", L, W.chain(3, 9), True, W.chi_matrix(ab=25 / 12, bs=35 / 12), tau=0.8,
                      noise=0.005, seed=seed, phi_p=0.12, precision="fp64")


LB_CASES = [
    ("bgk_tau0.8_17x5x9", lambda: small_melt(L=(17, 5, 9)).with_(tau=0.8)),
    ("mrt_9x7x11", lambda: small_melt(L=(9, 7, 11)).with_(lb="mrt", gammas=(0.3, -0.2, 0.1))),
]


@pytest.mark.parametrize("name,make", LB_CASES, ids=[c[0] for c in LB_CASES])
def test_lb_noise_parity(hsf, orc, name, make):
    """Three forced LB steps with mode noise (generator steps 7, 8, 9)."""
    wl = make()
    say(f"[lb noise] {name}")
    rng = np.random.default_rng(1)
    n = orc.lb_rest_state(osys(orc, wl)) * (1 + 0.02 * rng.uniform(-1, 1, size=(19,) + wl.shape))
    n = np.ascontiguousarray(n)
    f = np.ascontiguousarray(1e-3 * rng.uniform(-1, 1, size=(3,) + wl.shape))
    ctx = hsf.Context(wl)
    ctx.set_noise(cd=False, lb=True, omega=OMEGA, seed=1234, step=7)
    ctx.set_lb(n.ravel())
    ctx.lb_advance(3, f.ravel())
    assert ctx.noise_step() == 10
    got = ctx.get_lb().reshape(n.shape)
    ref = n
    plain = n
    for k in range(3):
        ref, rref, uref = orc.lb_step(osys(orc, wl, noise=2, omega=OMEGA, seed=1234, step=7 + k), ref, f)
        plain, _, _ = orc.lb_step(osys(orc, wl), plain, f)
    e = np.max(np.abs(got - ref))
    say(f"  max |dn| {e:.2e}; noise moved populations by {np.max(np.abs(ref - plain)):.2e}")
    assert np.max(np.abs(ref - plain)) > 1e-5
    assert e < 1e-14
    rho, u = ctx.get_flow()
    assert np.max(np.abs(rho.reshape(rref.shape) - rref)) < 1e-14
    assert np.max(np.abs(u.reshape(uref.shape) - uref)) < 1e-15
    assert abs(got.sum() / n.sum() - 1) < 1e-14


def test_cd_noise_parity(hsf, orc):
    """One convection-diffusion update with composition noise, solution (3 species)."""
    wl = small_solution(L=(10, 7, 12))
    rng = np.random.default_rng(2)
    phi = W.initial_composition(wl)
    mu = rng.standard_normal((3,) + wl.shape)
    u = 0.05 * rng.standard_normal((3,) + wl.shape)
    ctx = hsf.Context(wl)
    ctx.set_noise(cd=True, lb=False, omega=OMEGA, seed=99, step=41)
    ctx.set_densities(phi.ravel())
    ctx.cd_advance(mu.ravel(), u.ravel())
    assert ctx.noise_step() == 42
    got = ctx.get_densities().reshape(phi.shape)
    ref = orc.cd_update(osys(orc, wl, noise=1, omega=OMEGA, seed=99, step=41), phi, mu, u)
    plain = orc.cd_update(osys(orc, wl), phi, mu, u)
    e = np.max(np.abs(got - ref))
    say(f"[cd noise] max |dphi| {e:.2e}; noise moved densities by {np.max(np.abs(ref - plain)):.2e}")
    assert np.max(np.abs(ref - plain)) > 1e-4
    assert e < 1e-15
    assert np.max(np.abs(got.sum(axis=(1, 2, 3)) / phi.sum(axis=(1, 2, 3)) - 1)) < 1e-13


def test_noise_batched_replicas(hsf, orc):
    """Two replicas of different boxes in one context: replica r draws with key word r."""
    wls = [small_solution(L=(10, 7, 12), seed=3), small_solution(L=(8, 9, 5), seed=4)]
    say("[noise batched]")
    rng = np.random.default_rng(3)
    ctx = hsf.Context(wls)
    ctx.set_noise(cd=True, lb=True, omega=OMEGA, seed=5, step=0)
    phis = [W.initial_composition(w) for w in wls]
    mus = [rng.standard_normal((3,) + w.shape) for w in wls]
    ns = [np.ascontiguousarray(orc.lb_rest_state(osys(orc, w)) * (1 + 0.02 * rng.uniform(-1, 1, (19,) + w.shape)))
          for w in wls]
    ctx.set_densities(np.concatenate([p.ravel() for p in phis]))
    ctx.set_lb(np.concatenate([n.ravel() for n in ns]))
    ctx.lb_advance(1)
    ctx.cd_advance(np.concatenate([m.ravel() for m in mus]))
    got_n = ctx.get_lb()
    got_p = ctx.get_densities()
    off_n = off_p = 0
    for r, wl in enumerate(wls):
        ref_n, _, _ = orc.lb_step(osys(orc, wl, noise=2, omega=OMEGA, seed=5, rep=r, step=0), ns[r])
        ref_p = orc.cd_update(osys(orc, wl, noise=1, omega=OMEGA, seed=5, rep=r, step=1), phis[r], mus[r])
        gn = got_n[off_n:off_n + ref_n.size].reshape(ref_n.shape)
        gp = got_p[off_p:off_p + ref_p.size].reshape(ref_p.shape)
        off_n += ref_n.size
        off_p += ref_p.size
        say(f"  replica {r} L={wl.L}: |dn| {np.max(np.abs(gn - ref_n)):.2e} |dphi| {np.max(np.abs(gp - ref_p)):.2e}")
        assert np.max(np.abs(gn - ref_n)) < 1e-14
        assert np.max(np.abs(gp - ref_p)) < 1e-15


@pytest.mark.parametrize("lb", ["bgk", "mrt"])
def test_noisy_coupled_trajectory_fp64(hsf, orc, lb):
    """16^3 A4B4 melt with both noises (Omega = 400) for 10 coupled steps; the oracle
    takes the GPU's iteration counts (mirror mode) and the same generator steps."""
    wl = small_melt()
    if lb == "mrt":
        wl = wl.with_(lb="mrt", gammas=W.mrt_gammas(0.8, 1.2, 0.0))
    say(f"[noisy trajectory] melt16 a4b4 fp64 {lb}")
    sysw = osys(orc, wl, noise=3, omega=OMEGA, seed=77)
    phi = W.initial_composition(wl)
    ctx = hsf.Context(wl)
    ctx.set_noise(cd=True, lb=True, omega=OMEGA, seed=77, step=0)
    ctx.set_densities(phi.ravel())
    w = -np.log(phi / phi.mean(axis=(1, 2, 3), keepdims=True))
    ctx.set_fields(w.ravel())
    n = orc.lb_rest_state(sysw)
    for k in range(10):
        st, _ = ctx.step(1, tol=wl.tol, max_iter=1000)
        sysw.step = k
        phi, w, n, st_ref, u, rho, rc = orc.step(sysw, phi, w, n, tol=wl.tol, max_iter=1000,
                                                 fixed_iters=st[0]["iterations"])
        got = ctx.get_densities().reshape(phi.shape)
        e = relerr(got, phi)
        assert e < 1e-10, (k, e)
    assert ctx.noise_step() == 10
    ng = ctx.get_lb().reshape(n.shape)
    say(f"  densities rel err {e:.2e}; max |dn| {np.max(np.abs(ng - n)):.2e}")
    assert np.max(np.abs(ng - n)) < 1e-13


def test_gpu_lb_equipartition(hsf):
    """The GPU's fluctuating LB at rest reaches <u_a^2> = kT / rho and
    <delta rho^2> = rho kT / c_s^2 with kT = dt^2 / Omega (32^3, BGK tau 1, 400 steps)."""
    wl = small_melt(L=(32, 32, 32))
    dt, omega = wl.dt, 1.0
    kT = dt * dt / omega
    ctx = hsf.Context(wl)
    ctx.set_noise(cd=False, lb=True, omega=omega, seed=3)
    ctx.lb_advance(100)
    u2 = r2 = 0.0
    for _ in range(30):
        ctx.lb_advance(10)
        rho, u = ctx.get_flow()
        u2 += (u * u).mean()
        r2 += ((rho - 1.0) ** 2).mean()
    u2 /= 30
    r2 /= 30
    say(f"[gpu equipartition] <u^2>/kT {u2 / kT:.4f}, <drho^2>/(3 kT) {r2 / (3 * kT):.4f}")
    assert abs(u2 / kT - 1) < 0.03 and abs(r2 / (3 * kT) - 1) < 0.03
