"""ctypes front end of the FP64 CPU oracle (``hsf_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the library under test never
does.  It shares no code with the HIP library: it loads its own shared object,
built from ``hsf_oracle.c`` by :func:`build` with plain ``gcc``.

Array conventions: fields and densities are float64 arrays of shape
``(species, Lz, Ly, Lx)`` (x fastest); LB populations ``(19, Lz, Ly, Lx)``;
vectors ``(3, Lz, Ly, Lx)``.  Species order: A, B, then S when present.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hsf_oracle.c")
_LIB = os.path.join(_HERE, "libhsf_oracle.so")
MAX_BEADS = 64


_LIB_OMP = os.path.join(_HERE, "libhsf_oracle_omp.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, so the arithmetic is
    exactly the expressions written in the source), and its OpenMP build, whose
    site loops run over z-planes in parallel with bit-identical results (used only
    to time the oracle on all host cores)."""
    for lib, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
            tmp = lib + ".tmp"
            subprocess.check_call([
                "gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math", *extra,
                "-shared", "-fPIC", "-std=c99", "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, lib)
    return _LIB


class _Sys(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_int), ("Ly", ctypes.c_int), ("Lz", ctypes.c_int),
        ("N", ctypes.c_int), ("types", ctypes.c_int * MAX_BEADS),
        ("n_poly", ctypes.c_int), ("has_solvent", ctypes.c_int),
        ("c", ctypes.c_double * 4), ("chi", (ctypes.c_double * 3) * 3),
        ("kappa", ctypes.c_double), ("dt", ctypes.c_double), ("tau", ctypes.c_double),
        ("gamma_b", ctypes.c_double), ("gamma_s", ctypes.c_double),
        ("gamma_ghost", ctypes.c_double), ("lb_mode", ctypes.c_int), ("hydro", ctypes.c_int),
        ("precond", ctypes.c_int),
        ("noise", ctypes.c_int), ("omega", ctypes.c_double), ("seed", ctypes.c_ulonglong),
        ("rep", ctypes.c_ulonglong), ("step", ctypes.c_ulonglong),
    ]


class InvertStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("evaluations", ctypes.c_int),
                ("restarts", ctypes.c_int), ("residual", ctypes.c_double),
                ("converged", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_libs = {}
_P = ctypes.POINTER(ctypes.c_double)


def set_parallel(on: bool) -> int:
    """Route every oracle call through the OpenMP build (on) or the plain one; returns
    the number of threads the site loops then use."""
    global _lib
    _lib = _open(_LIB_OMP if on else _LIB)
    return _lib.orc_threads()


def _load():
    global _lib
    if _lib is None:
        _lib = _open(_LIB)
    return _lib


def _open(path):
    if path not in _libs:
        if not os.path.exists(path):
            build(force=False)
        lib = ctypes.CDLL(path)
        S = ctypes.POINTER(_Sys)
        lib.orc_stencil_weights.argtypes = [ctypes.c_double, _P]
        lib.orc_sigma.argtypes = [S, _P, _P]
        lib.orc_evaluate.argtypes = [S, _P, ctypes.c_double, ctypes.c_double, _P, _P, _P]
        lib.orc_evaluate.restype = ctypes.c_int
        lib.orc_log_q.argtypes = [S, _P]
        lib.orc_log_q.restype = ctypes.c_double
        lib.orc_invert.argtypes = [S, _P, _P, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(InvertStats)]
        lib.orc_invert.restype = ctypes.c_int
        lib.orc_mu_force.argtypes = [S, _P, _P, _P, _P]
        lib.orc_lb_step.argtypes = [S, _P, _P, _P, _P, _P]
        lib.orc_lb_equilibrium.argtypes = [ctypes.c_double, _P, _P]
        lib.orc_lb_velocity.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        lib.orc_free_energy.argtypes = [S, _P, _P]
        lib.orc_free_energy.restype = ctypes.c_double
        lib.orc_order_params.argtypes = [S, _P, _P, _P]
        lib.orc_order_params.restype = None
        lib.orc_mrt_basis.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.orc_mrt_basis.restype = ctypes.c_double
        lib.orc_cd_update.argtypes = [S, _P, _P, _P, _P]
        lib.orc_step.argtypes = [S, _P, _P, _P, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(InvertStats), _P, _P]
        lib.orc_step.restype = ctypes.c_int
        U64 = ctypes.POINTER(ctypes.c_ulonglong)
        lib.orc_philox4x64.argtypes = [U64, U64, U64]
        lib.orc_philox4x64.restype = None
        lib.orc_normals.argtypes = [S, ctypes.c_ulonglong, ctypes.c_ulonglong, _P]
        lib.orc_normals.restype = None
        lib.orc_threads.argtypes = []
        lib.orc_threads.restype = ctypes.c_int
        _libs[path] = lib
    return _libs[path]


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_P)


def stencil_weights(a: float) -> np.ndarray:
    c = np.zeros(4)
    _load().orc_stencil_weights(float(a), _ptr(c))
    return c


@dataclass
class System:
    """Parameters of one periodic system (lattice units, kT = 1)."""
    L: tuple                      # (Lx, Ly, Lz)
    types: list                   # species of beads 1..N (0 = A, 1 = B)
    has_solvent: bool = False
    c: np.ndarray = None          # stencil weights (centre, face, edge, corner)
    a: float = 1.1543             # statistical segment length, used when c is None
    chi: np.ndarray = field(default_factory=lambda: np.zeros((3, 3)))
    kappa: float = 10.0
    dt: float = 0.01
    tau: float = 1.0
    gamma_b: float = 0.0
    gamma_s: float = 0.0
    gamma_ghost: float = 0.0
    lb_mode: int = 0
    hydro: bool = True
    precond: bool = False
    noise: int = 0                # bit 0: composition noise (eq. 5), bit 1: LB mode noise (eq. 13)
    omega: float = 400.0          # noise scaling parameter Omega = h^3 / v0
    seed: int = 0                 # generator key word 0
    rep: int = 0                  # generator key word 1 (replica index)
    step: int = 0                 # generator counter word 1 (time step)

    @property
    def V(self):
        return int(np.prod(self.L))

    @property
    def N(self):
        return len(self.types)

    @property
    def nsp(self):
        return 3 if self.has_solvent else 2

    @property
    def shape(self):
        Lx, Ly, Lz = self.L
        return (Lz, Ly, Lx)

    def _c(self):
        if self.c is None:
            _load()
            return stencil_weights(self.a)
        return np.asarray(self.c, dtype=np.float64)

    def cstruct(self):
        s = _Sys()
        s.Lx, s.Ly, s.Lz = (int(v) for v in self.L)
        s.N = self.N
        assert 1 <= self.N <= MAX_BEADS
        for i, t in enumerate(self.types):
            s.types[i] = int(t)
        s.n_poly = 2
        s.has_solvent = int(bool(self.has_solvent))
        c = self._c()
        for k in range(4):
            s.c[k] = float(c[k])
        chi = np.asarray(self.chi, dtype=np.float64)
        for i in range(3):
            for j in range(3):
                s.chi[i][j] = float(chi[i, j])
        s.kappa, s.dt, s.tau = float(self.kappa), float(self.dt), float(self.tau)
        s.gamma_b, s.gamma_s, s.gamma_ghost = float(self.gamma_b), float(self.gamma_s), float(self.gamma_ghost)
        s.lb_mode = int(self.lb_mode)
        s.hydro = int(bool(self.hydro))
        s.precond = int(bool(self.precond))
        s.noise = int(self.noise)
        s.omega = float(self.omega)
        s.seed, s.rep, s.step = int(self.seed), int(self.rep), int(self.step)
        return s


def _arr(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.shape == shape, (a.shape, shape)
    return a


def sigma(sys: System, f):
    f = _arr(f, sys.shape)
    out = np.empty_like(f)
    s = sys.cstruct()
    _load().orc_sigma(ctypes.byref(s), _ptr(f), _ptr(out))
    return out


def evaluate(sys: System, w, phibar_p=1.0, phibar_s=0.0, with_qs=False):
    """Densities phi[w]; returns (phi, Q) or (phi, Q, Qs)."""
    w = _arr(w, (sys.nsp,) + sys.shape)
    phi = np.empty_like(w)
    q = ctypes.c_double(0.0)
    qs = np.zeros(sys.N)
    s = sys.cstruct()
    rc = _load().orc_evaluate(ctypes.byref(s), _ptr(w), float(phibar_p), float(phibar_s),
                              _ptr(phi), ctypes.byref(q), _ptr(qs))
    if rc != 0:
        raise MemoryError("oracle evaluate failed")
    return (phi, q.value, qs) if with_qs else (phi, q.value)


def free_energy(sys: System, w, phi):
    """Free-energy density v0 F / (kT V) of eq. 1 at fields w and volume fractions phi."""
    w = _arr(w, (sys.nsp,) + sys.shape)
    phi = _arr(phi, (sys.nsp,) + sys.shape)
    s = sys.cstruct()
    return _load().orc_free_energy(ctypes.byref(s), _ptr(w), _ptr(phi))


def order_params(sys: System, phi):
    """(S of the melt, S of the solution) of the composition phi."""
    phi = _arr(phi, (sys.nsp,) + sys.shape)
    a, b = ctypes.c_double(0.0), ctypes.c_double(0.0)
    s = sys.cstruct()
    _load().orc_order_params(ctypes.byref(s), _ptr(phi), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def log_q(sys: System, w):
    w = _arr(w, (sys.nsp,) + sys.shape)
    s = sys.cstruct()
    return _load().orc_log_q(ctypes.byref(s), _ptr(w))


def invert(sys: System, phit, w0, tol=1e-8, max_iter=1000, fixed_iters=0):
    """Fields w with phi[w] = phit; returns (w, stats dict, status)."""
    phit = _arr(phit, (sys.nsp,) + sys.shape)
    w = _arr(w0, (sys.nsp,) + sys.shape).copy()
    st = InvertStats()
    s = sys.cstruct()
    rc = _load().orc_invert(ctypes.byref(s), _ptr(phit), _ptr(w), float(tol), int(max_iter),
                            int(fixed_iters), ctypes.byref(st))
    if rc < 0:
        raise MemoryError("oracle invert failed")
    return w, st.as_dict(), rc


def mu_force(sys: System, phi, w):
    phi = _arr(phi, (sys.nsp,) + sys.shape)
    w = _arr(w, (sys.nsp,) + sys.shape)
    mu = np.empty_like(phi)
    f = np.empty((3,) + sys.shape)
    s = sys.cstruct()
    _load().orc_mu_force(ctypes.byref(s), _ptr(phi), _ptr(w), _ptr(mu), _ptr(f))
    return mu, f


def lb_step(sys: System, n, f=None):
    """One LB collide+stream step; returns (n_new, rho, u)."""
    n = _arr(n, (19,) + sys.shape)
    f = None if f is None else _arr(f, (3,) + sys.shape)
    nout = np.empty_like(n)
    rho = np.empty(sys.shape)
    u = np.empty((3,) + sys.shape)
    s = sys.cstruct()
    _load().orc_lb_step(ctypes.byref(s), _ptr(n), _ptr(f), _ptr(nout), _ptr(rho), _ptr(u))
    return nout, rho, u


def lb_equilibrium(rho, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(19)
    _load().orc_lb_equilibrium(float(rho), _ptr(u), _ptr(out))
    return out


def lb_velocities():
    _load()
    out = np.zeros((19, 3), dtype=np.int64)
    c = (ctypes.c_int * 3)()
    for i in range(19):
        _lib.orc_lb_velocity(i, c)
        out[i] = list(c)
    return out


def mrt_basis():
    _load()
    return np.array([[_lib.orc_mrt_basis(k, i) for i in range(19)] for k in range(19)])


def cd_update(sys: System, phi, mu, u=None):
    phi = _arr(phi, (sys.nsp,) + sys.shape)
    mu = _arr(mu, (sys.nsp,) + sys.shape)
    u = None if u is None else _arr(u, (3,) + sys.shape)
    out = np.empty_like(phi)
    s = sys.cstruct()
    _load().orc_cd_update(ctypes.byref(s), _ptr(phi), _ptr(mu), _ptr(u), _ptr(out))
    return out


def step(sys: System, phi, w, n=None, tol=1e-8, max_iter=1000, fixed_iters=0):
    """One coupled step; returns (phi_new, w_new, n_new, stats, u, rho, status)."""
    phi = _arr(phi, (sys.nsp,) + sys.shape).copy()
    w = _arr(w, (sys.nsp,) + sys.shape).copy()
    n = None if n is None else _arr(n, (19,) + sys.shape).copy()
    u = np.zeros((3,) + sys.shape)
    rho = np.zeros(sys.shape)
    st = InvertStats()
    s = sys.cstruct()
    rc = _load().orc_step(ctypes.byref(s), _ptr(phi), _ptr(w), _ptr(n), float(tol), int(max_iter),
                          int(fixed_iters), ctypes.byref(st), _ptr(u), _ptr(rho))
    if rc < 0:
        raise MemoryError("oracle step failed")
    return phi, w, n, st.as_dict(), u, rho, rc


def philox4x64(ctr, key):
    """Philox4x64-10 of the 4-word counter and 2-word key (four 64-bit words)."""
    c = (ctypes.c_ulonglong * 4)(*[int(v) for v in ctr])
    k = (ctypes.c_ulonglong * 2)(*[int(v) for v in key])
    o = (ctypes.c_ulonglong * 4)()
    _load().orc_philox4x64(c, k, o)
    return [int(v) for v in o]


def normals(sys: System, site, purpose):
    """The four standard normal numbers of (site, purpose) at the system's step."""
    z = np.empty(4)
    s = sys.cstruct()
    _load().orc_normals(ctypes.byref(s), int(site), int(purpose), _ptr(z))
    return z


def lb_rest_state(sys: System, rho0=1.0):
    """Populations at rest with density rho0 (equilibrium of eq. 11 at u = 0)."""
    neq = lb_equilibrium(rho0, np.zeros(3))
    return np.ascontiguousarray(np.broadcast_to(neq[:, None, None, None], (19,) + sys.shape).copy())


# ---------------------------------------------------------------------------
# Crank-Nicolson diffusion (section 2: the diffusive part of eq. 3 is integrated
# with the implicit Crank-Nicolson scheme, convection with explicit two-step
# Lax-Wendroff).  With B(phi, mu) the diffusive rate div(phi grad mu) of the
# conservative face fluxes of orc_cd_update (M = 1) and J^C the convective flux,
#   phi^{n+1} = phi^n + dt/2 [B(phi^n, mu^n) + B(phi^{n+1}, mu^{n+1})] - div J^C(phi^n, u^n) + xi^n,
# where mu^{n+1} = mu[phi^{n+1}] requires the self-consistent fields of phi^{n+1}.
# The unknowns are those fields: phi^{n+1} = phi[w], and
#   F(w) = phi[w] - dt/2 B(phi[w], mu(phi[w], w)) - rhs = 0,
#   rhs = phi^n + dt/2 B(phi^n, mu^n) - div J^C + xi^n.
# This oracle solves F = 0 by Newton's method with the full Jacobian by forward
# differences (one column per unknown) and a least-squares solve (the fields'
# per-species constants are a null space of F); it is meant for small boxes.
# ---------------------------------------------------------------------------

def _diffusive_rate(sys: System, phi, mu):
    """B(phi, mu) = div(phi grad mu) of the explicit step's face fluxes (no flow, no noise)."""
    s1 = replace(sys, dt=1.0, noise=0)
    return cd_update(s1, phi, mu) - _arr(phi, (sys.nsp,) + sys.shape)


def cn_residual(sys: System, w, rhs, phibar_p, phibar_s):
    """F(w) and phi[w] of the Crank-Nicolson equation."""
    p, _ = evaluate(sys, w, phibar_p, phibar_s)
    mu, _ = mu_force(sys, p, w)
    return p - 0.5 * sys.dt * _diffusive_rate(sys, p, mu) - rhs, p


def cn_step(sys: System, phi, w, n=None, tol=1e-12, max_newton=20, invert_tol=1e-13, h=1e-7):
    """One coupled step with Crank-Nicolson diffusion.  Order as in `step`: invert
    phi^n, mu^n and the force, the LB step (hydro on, n given) giving u^n, then the CD
    update, here implicit.  Returns (phi^{n+1}, w^{n+1}, n^{n+1}, info) with
    phi^{n+1} = phi[w^{n+1}] and info = {"newton": iterations, "residual": max |F|,
    "evaluations": density evaluations of the Newton solve}."""
    shape = (sys.nsp,) + sys.shape
    phi = _arr(phi, shape).copy()
    w, st, rc = invert(sys, phi, w, tol=invert_tol, max_iter=20000)
    if rc != 0:
        raise RuntimeError(f"inversion of phi^n failed: {st}")
    pbar_p = phi[:2].sum(0).mean()
    pbar_s = phi[2].mean() if sys.has_solvent else 0.0
    mu, f = mu_force(sys, phi, w)
    u = None
    if sys.hydro and n is not None:
        n, _, u = lb_step(sys, n, f)
    full = cd_update(sys, phi, mu, u)                      # phi + dt B - div J^C + xi
    rhs = full - 0.5 * sys.dt * _diffusive_rate(sys, phi, mu)
    evals = 0
    x = w.ravel().copy()
    for it in range(max_newton + 1):
        F, p = cn_residual(sys, x.reshape(shape), rhs, pbar_p, pbar_s)
        evals += 1
        res = np.max(np.abs(F))
        if res <= tol or it == max_newton:
            break
        Fv = F.ravel()
        J = np.empty((Fv.size, x.size))
        for j in range(x.size):
            xp = x.copy()
            xp[j] += h
            J[:, j] = (cn_residual(sys, xp.reshape(shape), rhs, pbar_p, pbar_s)[0].ravel() - Fv) / h
        evals += x.size
        dx = np.linalg.lstsq(J, -Fv, rcond=1e-12)[0]
        x = x + dx
    return p, x.reshape(shape), n, {"newton": it, "residual": res, "evaluations": evals}
