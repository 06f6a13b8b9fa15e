"""Seeded synthetic workloads: parameter sets and initial compositions.

This module holds parameters and random inputs only, none of the method's
arithmetic.  The test suite and the benchmark draw inputs here and hand the
same arrays to the GPU library and to the CPU oracle.

Parameter readings (lattice units, kT = 1, h = 1):
  * chi_IJ = (chi N) / N with N the copolymer length;
  * kappa_H v0 / kT = 10 and a = 1.1543 (paper section 2, model parameters);
  * explicit time step dt = 0.01 (the explicit diffusion update is stable
    below about 0.015 at these parameters);
  * initial compositions: bulk fractions plus seeded uniform noise with its
    mean removed, so each species' total is exactly the bulk value and the
    A:B ratio of the target is exactly n:m.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

A, B, S = 0, 1, 2


def chain(n_a: int, n_b: int):
    """Bead species of an A_n B_m diblock, bead 1 first."""
    return [A] * n_a + [B] * n_b


@dataclass
class Workload:
    name: str
    L: tuple                     # (Lx, Ly, Lz)
    types: list                  # bead species, bead 1 first
    has_solvent: bool
    chi: np.ndarray              # 3x3 symmetric Flory-Huggins matrix
    tau: float                   # BGK relaxation time of the LB fluid
    noise: float                 # amplitude of the initial uniform noise
    seed: int
    phi_p: float = 1.0           # copolymer volume fraction (1 for melts)
    precision: str = "fp64"      # propagator precision: fp64 | fp32
    tol: float = 1e-8            # inversion residual
    steps: int = 100
    dt: float = 0.01
    kappa: float = 10.0
    a: float = 1.1543
    hydro: bool = True
    lb: str = "bgk"              # LB collision: "bgk" (tau) or "mrt" (gammas)
    gammas: tuple = (0.0, 0.0, 0.0)   # MRT eigenvalues (shear, bulk, ghost)
    extra: dict = field(default_factory=dict)

    @property
    def N(self):
        return len(self.types)

    @property
    def nsp(self):
        return 3 if self.has_solvent else 2

    @property
    def V(self):
        return int(np.prod(self.L))

    @property
    def shape(self):
        Lx, Ly, Lz = self.L
        return (Lz, Ly, Lx)

    def with_(self, **kw):
        return replace(self, **kw)


def mrt_gammas(tau, tau_bulk=None, ghost=0.0):
    """MRT eigenvalues with the shear viscosity of the BGK relaxation time tau
    (gamma_s = 1 - 1/tau, nu = (tau - 1/2)/3), the bulk one from tau_bulk (default
    tau) and the kinetic modes at `ghost` (0: relaxed completely every step)."""
    tb = tau if tau_bulk is None else tau_bulk
    return (1.0 - 1.0 / tau, 1.0 - 1.0 / tb, ghost)


def chi_matrix(ab=0.0, as_=0.0, bs=0.0):
    m = np.zeros((3, 3))
    m[A, B] = m[B, A] = ab
    m[A, S] = m[S, A] = as_
    m[B, S] = m[S, B] = bs
    return m


def melt16_a4b4():
    """16^3 symmetric A4B4 melt, chi N = 20, FP64, tau 1.0, residual 1e-8, 100 steps."""
    return Workload("melt16_a4b4", (16, 16, 16), chain(4, 4), False, chi_matrix(ab=20 / 8),
                    tau=1.0, noise=0.01, seed=0, precision="fp64", tol=1e-8, steps=100)


def melt64_a8b8(tau=0.6, precision="fp32"):
    """64^3 symmetric A8B8 melt, chi N = 20, tau 0.6 or 1.5, FP32 or FP64 propagators."""
    return Workload("melt64_a8b8", (64, 64, 64), chain(8, 8), False, chi_matrix(ab=20 / 16),
                    tau=tau, noise=0.01, seed=0, precision=precision,
                    tol=1e-6 if precision == "fp32" else 1e-8, steps=2000)


def melt192_a8b8(precision="fp32"):
    """192^3 A8B8 melt, chi N = 20, tau 1.0: a box whose propagator store (16 x 7.1 M
    sites, 453 MB in FP32) and LB populations (2 x 1.08 GB) exceed the on-package caches,
    so the kernels stream from HBM."""
    return Workload("melt192_a8b8", (192, 192, 192), chain(8, 8), False, chi_matrix(ab=20 / 16),
                    tau=1.0, noise=0.01, seed=0, precision=precision,
                    tol=1e-6 if precision == "fp32" else 1e-8, steps=100)


def melt96_a4b12(hydro=True):
    """96^3 asymmetric A4B12 melt, chi N = 25, tau 1.0, FP32, noise 0.005."""
    return Workload("melt96_a4b12", (96, 96, 96), chain(4, 12), False, chi_matrix(ab=25 / 16),
                    tau=1.0, noise=0.005, seed=0, precision="fp32", tol=1e-6, steps=5000,
                    hydro=hydro)


def batch48_a3b9s(n_rep=48, meta_seed=1234):
    """Replicas of an A3B9 + S solution, phi_p = 0.1, box drawn from {32,48,64}^3,
    chi_AB N ~ U[15, 30], chi_AS = 0, chi_BS N = 30, tau 1.0, FP32."""
    rng = np.random.Generator(np.random.PCG64(meta_seed))
    sizes = rng.choice([32, 48, 64], size=n_rep)
    chins = rng.uniform(15.0, 30.0, size=n_rep)
    out = []
    for r in range(n_rep):
        L = int(sizes[r])
        out.append(Workload(f"batch48_a3b9s[{r}]", (L, L, L), chain(3, 9), True,
                            chi_matrix(ab=float(chins[r]) / 12, bs=30 / 12),
                            tau=1.0, noise=0.005, seed=r, phi_p=0.1, precision="fp32",
                            tol=1e-6, steps=100, extra={"chiN_AB": float(chins[r])}))
    return out


def vesicle128_a3b9s(L=128):
    """128^3 A3B9 + S solution, phi_p = 0.12, chi_AB N = 25, chi_BS N = 35, tau 0.8, FP32, residual 1e-6."""
    return Workload(f"vesicle{L}_a3b9s", (L, L, L), chain(3, 9), True,
                    chi_matrix(ab=25 / 12, bs=35 / 12), tau=0.8, noise=0.005, seed=0,
                    phi_p=0.12, precision="fp32", tol=1e-6, steps=3000)


def initial_composition(wl: Workload) -> np.ndarray:
    """Volume fractions [species][Lz][Ly][Lx] of the quench's initial state.

    Melt: phi_A = f + eta, phi_B = 1 - phi_A.  Solution: phi_A, phi_B = bulk
    fraction + independent noise, phi_S = 1 - phi_A - phi_B.  Noise is
    uniform on (-noise, noise) from numpy's PCG64 with the workload's seed,
    with its mean removed.
    """
    rng = np.random.Generator(np.random.PCG64(wl.seed))
    nA = sum(1 for t in wl.types if t == A)
    f = nA / wl.N

    def eta():
        e = rng.uniform(-wl.noise, wl.noise, size=wl.shape)
        return e - e.mean()

    phi = np.empty((wl.nsp,) + wl.shape)
    if not wl.has_solvent:
        phi[A] = f + eta()
        phi[B] = 1.0 - phi[A]
    else:
        phi[A] = wl.phi_p * f + eta()
        phi[B] = wl.phi_p * (1.0 - f) + eta()
        phi[S] = 1.0 - phi[A] - phi[B]
    return phi


def random_fields(shape_sp, seed, amplitude=1.0, smooth=0):
    """Random fields w [species][Lz][Ly][Lx], uniform on (-amplitude, amplitude)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.uniform(-amplitude, amplitude, size=shape_sp)
    for _ in range(smooth):
        w = (w + np.roll(w, 1, -1) + np.roll(w, -1, -1) + np.roll(w, 1, -2) + np.roll(w, -1, -2)
             + np.roll(w, 1, -3) + np.roll(w, -1, -3)) / 7.0
    return np.ascontiguousarray(w)
