"""Python binding of the C ABI in ``include/hsf.h`` (argument marshalling only).

Every step of the method runs in the HIP library ``libhsf.so``; this module
converts arguments.  Data arguments are numpy arrays (host memory, copied
synchronously) or torch tensors on the GPU (device memory, ordered on the
context's stream).  All arrays are float64, C-contiguous, in the layouts of
the header: fields ``(species, Lz, Ly, Lx)`` per replica, replicas
concatenated.

If the shared library is missing the import of :func:`load` raises: there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhsf.so")
MAX_BEADS = 64

HSF_OK, HSF_EINVAL, HSF_ENOMEM, HSF_EHIP, HSF_ENOCONV, HSF_ENONFINITE = 0, -1, -2, -3, -4, -5
HOST, DEVICE = 0, 1
FP64, FP32 = 0, 1
WARM_CURRENT, WARM_LOCAL = 0, 1

EXPORTED = [
    "hsf_create", "hsf_destroy", "hsf_last_error", "hsf_set_stream", "hsf_total_sites",
    "hsf_site_offset", "hsf_field_offset", "hsf_num_species", "hsf_set_fields", "hsf_get_fields",
    "hsf_set_densities", "hsf_get_densities", "hsf_evaluate", "hsf_evaluate_static", "hsf_observables",
    "hsf_invert", "hsf_mu_force",
    "hsf_set_lb", "hsf_get_lb", "hsf_lb_advance", "hsf_get_flow", "hsf_cd_advance", "hsf_step",
    "hsf_set_hydro", "hsf_set_noise", "hsf_get_noise_step", "hsf_set_integrator", "hsf_get_cn_stats",
    "hsf_state_size", "hsf_get_state", "hsf_set_state", "hsf_set_timing", "hsf_get_timing", "hsf_set_tile", "hsf_get_tile", "hsf_autotune",
    "hsf_set_solver", "hsf_get_work", "hsf_set_warm", "hsf_net_create", "hsf_net_destroy",
    "hsf_net_last_error", "hsf_net_set_stream", "hsf_net_num_params", "hsf_net_set_params",
    "hsf_net_get_params", "hsf_net_set_input_norm", "hsf_net_set_output_scale", "hsf_net_forward", "hsf_net_loss_grad",
    "hsf_net_train_step", "hsf_attach_net", "hsf_set_net_gate", "hsf_paired_schedule", "hsf_net_make_sample",
    "hsf_net_channel_moments", "hsf_net_affine", "hsf_set_step_log", "hsf_read_step_log",
]
WARM_EXTRAP, WARM_NET, WARM_NET_DELTA, WARM_NET_EXTRAP = 2, 3, 4, 5
SOLVER_PRECOND, SOLVER_REFINE = 1, 2
LB_BGK, LB_MRT = 0, 1
NOISE_CD, NOISE_LB = 1, 2
CD_EXPLICIT, CD_CRANK_NICOLSON = 0, 1
K_PREP, K_FWD, K_BWD, K_LB, K_CD, K_PAIR, K_COUNT = 0, 1, 2, 3, 4, 5, 6
KERNEL_NAMES = ["prep", "fwd", "bwd", "lb", "cd", "pair"]


class HsfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hsf error {code}: {msg}")
        self.code = code


class CnStats(ctypes.Structure):
    _fields_ = [("newton", ctypes.c_int), ("krylov", ctypes.c_int), ("evaluations", ctypes.c_longlong),
                ("residual", ctypes.c_double), ("converged", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StepRecord(ctypes.Structure):
    _fields_ = [("step", ctypes.c_longlong), ("replica", ctypes.c_int), ("iterations", ctypes.c_int),
                ("evaluations", ctypes.c_int), ("converged", ctypes.c_int), ("residual", ctypes.c_double),
                ("ln_q", ctypes.c_double), ("amount", ctypes.c_double * 3), ("max_u", ctypes.c_double),
                ("ms_inversion", ctypes.c_double), ("ms_dynamics", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["amount"] = list(self.amount)
        return d


class Params(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_int), ("Ly", ctypes.c_int), ("Lz", ctypes.c_int),
        ("n_beads", ctypes.c_int), ("types", ctypes.c_int * MAX_BEADS),
        ("has_solvent", ctypes.c_int), ("a", ctypes.c_double), ("stencil", ctypes.c_double * 4),
        ("chi", (ctypes.c_double * 3) * 3), ("kappa", ctypes.c_double), ("dt", ctypes.c_double),
        ("tau", ctypes.c_double), ("hydro", ctypes.c_int), ("precision", ctypes.c_int),
        ("lb_mode", ctypes.c_int), ("gamma_s", ctypes.c_double), ("gamma_b", ctypes.c_double),
        ("gamma_ghost", ctypes.c_double),
    ]


class InvertStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("evaluations", ctypes.c_int),
                ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
                ("residual", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load ``libhsf.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with `python -m paper_1204_2088_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    C = ctypes.c_void_p  # hsf_ctx*
    I = ctypes.c_int
    sig = {
        "hsf_create": ([ctypes.POINTER(Params), I, ctypes.POINTER(C)], I),
        "hsf_destroy": ([C], None),
        "hsf_last_error": ([C], ctypes.c_char_p),
        "hsf_set_stream": ([C, P], I),
        "hsf_total_sites": ([C], ctypes.c_longlong),
        "hsf_site_offset": ([C, I], ctypes.c_longlong),
        "hsf_field_offset": ([C, I], ctypes.c_longlong),
        "hsf_num_species": ([C], I),
        "hsf_set_fields": ([C, P, I], I),
        "hsf_get_fields": ([C, P, I], I),
        "hsf_set_densities": ([C, P, I], I),
        "hsf_get_densities": ([C, P, I], I),
        "hsf_evaluate": ([C, P, P, I], I),
        "hsf_observables": ([C, P, P, P], I),
        "hsf_invert": ([C, ctypes.c_double, I, I, ctypes.POINTER(InvertStats)], I),
        "hsf_mu_force": ([C, P, P, I], I),
        "hsf_set_lb": ([C, P, I], I),
        "hsf_get_lb": ([C, P, I], I),
        "hsf_lb_advance": ([C, I, P, I], I),
        "hsf_get_flow": ([C, P, P, I], I),
        "hsf_cd_advance": ([C, P, P, I], I),
        "hsf_step": ([C, I, ctypes.c_double, I, ctypes.POINTER(InvertStats),
                      ctypes.POINTER(ctypes.c_longlong)], I),
        "hsf_set_hydro": ([C, I], I),
        "hsf_set_noise": ([C, I, ctypes.c_double, ctypes.c_ulonglong, ctypes.c_ulonglong], I),
        "hsf_get_noise_step": ([C, ctypes.POINTER(ctypes.c_ulonglong)], I),
        "hsf_set_integrator": ([C, I, ctypes.c_double, I, I], I),
        "hsf_state_size": ([C], ctypes.c_longlong),
        "hsf_get_state": ([C, P, ctypes.c_longlong], I),
        "hsf_set_state": ([C, P, ctypes.c_longlong], I),
        "hsf_get_cn_stats": ([C, ctypes.POINTER(CnStats)], I),
        "hsf_set_timing": ([C, I], I),
        "hsf_set_step_log": ([C, I], I),
        "hsf_read_step_log": ([C, ctypes.POINTER(StepRecord), I, ctypes.POINTER(I)], I),
        "hsf_set_solver": ([C, I], I),
        "hsf_set_warm": ([C, I], I),
        "hsf_net_create": ([I, I, ctypes.POINTER(ctypes.c_int), ctypes.c_ulonglong, ctypes.POINTER(C)], I),
        "hsf_net_destroy": ([C], None),
        "hsf_net_last_error": ([C], ctypes.c_char_p),
        "hsf_net_set_stream": ([C, P], I),
        "hsf_net_num_params": ([C], ctypes.c_longlong),
        "hsf_net_set_params": ([C, P, I], I),
        "hsf_net_get_params": ([C, P, I], I),
        "hsf_net_set_input_norm": ([C, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)], I),
        "hsf_net_set_output_scale": ([C, ctypes.POINTER(ctypes.c_float)], I),
        "hsf_net_forward": ([C, P, P, I, I, I], I),
        "hsf_net_loss_grad": ([C, P, P, I, I, ctypes.POINTER(ctypes.c_double), P, I], I),
        "hsf_net_train_step": ([C, P, P, I, I, ctypes.c_float, ctypes.POINTER(ctypes.c_double), I], I),
        "hsf_attach_net": ([C, C], I),
        "hsf_set_net_gate": ([C, I], I),
        "hsf_get_work": ([C, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double), I], I),
        "hsf_set_tile": ([C, ctypes.POINTER(ctypes.c_int)], I),
        "hsf_get_tile": ([C, ctypes.POINTER(ctypes.c_int)], I),
        "hsf_autotune": ([C, I, ctypes.POINTER(ctypes.c_double)], I),
        "hsf_get_timing": ([C, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)], I),
        "hsf_evaluate_static": ([ctypes.POINTER(Params), P, P, P, P, P], I),
        "hsf_paired_schedule": ([I, I, ctypes.POINTER(ctypes.c_int)], I),
        "hsf_net_make_sample": ([C, P, P, P, P, P, P, I, ctypes.c_longlong, I, P, P], I),
        "hsf_net_channel_moments": ([C, P, I, I, ctypes.c_longlong, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)], I),
        "hsf_net_affine": ([C, P, I, I, ctypes.c_longlong, ctypes.POINTER(ctypes.c_float),
                            ctypes.POINTER(ctypes.c_float)], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def params_from_workload(wl, precision=None):
    """hsf_params of one replica from a :class:`workloads.Workload`."""
    p = Params()
    p.Lx, p.Ly, p.Lz = (int(v) for v in wl.L)
    p.n_beads = wl.N
    for i, t in enumerate(wl.types):
        p.types[i] = int(t)
    p.has_solvent = int(bool(wl.has_solvent))
    p.a = float(wl.a)
    for k in range(4):
        p.stencil[k] = 0.0
    chi = np.asarray(wl.chi, dtype=np.float64)
    for i in range(3):
        for j in range(3):
            p.chi[i][j] = float(chi[i, j])
    p.kappa, p.dt, p.tau = float(wl.kappa), float(wl.dt), float(wl.tau)
    p.hydro = int(bool(wl.hydro))
    prec = precision or wl.precision
    p.precision = FP32 if prec == "fp32" else FP64
    p.lb_mode = LB_MRT if wl.lb == "mrt" else LB_BGK
    p.gamma_s, p.gamma_b, p.gamma_ghost = (float(v) for v in wl.gammas)
    return p


def _ptr32(a, n):
    """(pointer, where) of a float32 buffer holding at least n elements."""
    if a is None:
        return None, HOST
    if _is_torch(a):
        import torch
        assert a.dtype == torch.float32 and a.is_contiguous(), "need a contiguous float32 tensor"
        assert a.numel() >= n, (a.numel(), n)
        return ctypes.c_void_p(a.data_ptr()), (DEVICE if a.is_cuda else HOST)
    assert isinstance(a, np.ndarray) and a.dtype == np.float32 and a.flags.c_contiguous
    assert a.size >= n, (a.size, n)
    return ctypes.c_void_p(a.ctypes.data), HOST


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a, n):
    """(pointer, where) of a float64 buffer holding at least n elements."""
    if a is None:
        return None, HOST
    if _is_torch(a):
        import torch
        assert a.dtype == torch.float64 and a.is_contiguous(), "need a contiguous float64 tensor"
        assert a.numel() >= n, (a.numel(), n)
        return ctypes.c_void_p(a.data_ptr()), (DEVICE if a.is_cuda else HOST)
    assert isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous
    assert a.size >= n, (a.size, n)
    return ctypes.c_void_p(a.ctypes.data), HOST


STATIC_SCRATCH_BYTES = 64 << 20


def evaluate_static(wl, w, phi, phi_out, q_out, stream=None, precision=None):
    """hsf_evaluate_static: phi[w] and Q of one replica without a context and without any
    device allocation.  w, phi, phi_out: contiguous float64 CUDA tensors in the field
    layout; q_out: a float64 CUDA tensor of one element; stream: a torch stream (default:
    the current one).  Returns the library's status code (the work is only enqueued)."""
    import torch
    lib = load()
    n = (3 if wl.has_solvent else 2) * wl.V
    for a in (w, phi, phi_out):
        assert a.is_cuda and a.dtype == torch.float64 and a.is_contiguous() and a.numel() >= n
    assert q_out.is_cuda and q_out.dtype == torch.float64 and q_out.numel() >= 1
    s = (stream or torch.cuda.current_stream()).cuda_stream
    p = params_from_workload(wl, precision)
    return lib.hsf_evaluate_static(ctypes.byref(p), ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                                   ctypes.c_void_p(phi_out.data_ptr()), ctypes.c_void_p(q_out.data_ptr()),
                                   ctypes.c_void_p(s))


class Context:
    """A set of replicas on the current GPU (a single run is one replica)."""

    def __init__(self, workloads, precision=None, stream=None):
        lib = load()
        wls = workloads if isinstance(workloads, (list, tuple)) else [workloads]
        arr = (Params * len(wls))(*[params_from_workload(w, precision) for w in wls])
        h = ctypes.c_void_p()
        rc = lib.hsf_create(arr, len(wls), ctypes.byref(h))
        if rc != HSF_OK:
            raise HsfError(rc, "hsf_create failed")
        self._h = h
        self._lib = lib
        self.workloads = list(wls)
        self.n_rep = len(wls)
        self.nsp = lib.hsf_num_species(h)
        self.T = lib.hsf_total_sites(h)
        if stream is not None:
            self.set_stream(stream)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hsf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, ok=(HSF_OK,)):
        if rc not in ok:
            raise HsfError(rc, self._lib.hsf_last_error(self._h).decode())
        return rc

    # sizes
    def site_offset(self, r):
        return self._lib.hsf_site_offset(self._h, r)

    def field_offset(self, r):
        return self._lib.hsf_field_offset(self._h, r)

    def set_stream(self, stream):
        """stream: a torch.cuda.Stream, an integer hipStream_t, or None."""
        raw = getattr(stream, "cuda_stream", stream)
        self._check(self._lib.hsf_set_stream(self._h, ctypes.c_void_p(raw or 0)))

    # state transfer
    def _put(self, fn, a, n):
        p, where = _ptr(a, n)
        self._check(fn(self._h, p, where))

    def _get(self, fn, out, n, shape):
        if out is None:
            out = np.empty(shape, dtype=np.float64)
        p, where = _ptr(out, n)
        self._check(fn(self._h, p, where))
        return out

    def set_fields(self, w):
        self._put(self._lib.hsf_set_fields, w, self.nsp * self.T)

    def get_fields(self, out=None):
        return self._get(self._lib.hsf_get_fields, out, self.nsp * self.T, (self.nsp * self.T,))

    def set_densities(self, phi):
        self._put(self._lib.hsf_set_densities, phi, self.nsp * self.T)

    def get_densities(self, out=None):
        return self._get(self._lib.hsf_get_densities, out, self.nsp * self.T, (self.nsp * self.T,))

    def set_lb(self, n):
        self._put(self._lib.hsf_set_lb, n, 19 * self.T)

    def get_lb(self, out=None):
        return self._get(self._lib.hsf_get_lb, out, 19 * self.T, (19 * self.T,))

    # method
    def evaluate(self, out=None):
        """phi[w] (field layout) and Q per replica."""
        if out is None:
            out = np.empty(self.nsp * self.T)
        q = (ctypes.c_double * self.n_rep)()
        p, where = _ptr(out, self.nsp * self.T)
        self._check(self._lib.hsf_evaluate(self._h, p, q, where))
        return out, np.array(q[:])

    def observables(self):
        """Free-energy density (eq. 1), melt and solution order parameters per replica."""
        f = (ctypes.c_double * self.n_rep)()
        sm = (ctypes.c_double * self.n_rep)()
        ss = (ctypes.c_double * self.n_rep)()
        self._check(self._lib.hsf_observables(self._h, f, sm, ss))
        return np.array(f[:]), np.array(sm[:]), np.array(ss[:])

    def invert(self, tol=1e-8, max_iter=1000, warm=WARM_CURRENT, allow_noconv=False):
        st = (InvertStats * self.n_rep)()
        rc = self._lib.hsf_invert(self._h, float(tol), int(max_iter), int(warm), st)
        self._check(rc, (HSF_OK, HSF_ENOCONV) if allow_noconv else (HSF_OK,))
        return [s.as_dict() for s in st], rc

    def mu_force(self, mu=None, force=None):
        if mu is None:
            mu = np.empty(self.nsp * self.T)
        if force is None:
            force = np.empty(3 * self.T)
        pm, where = _ptr(mu, self.nsp * self.T)
        pf, _ = _ptr(force, 3 * self.T)
        self._check(self._lib.hsf_mu_force(self._h, pm, pf, where))
        return mu, force

    def lb_advance(self, n_steps, force=None):
        p, where = _ptr(force, 3 * self.T)
        self._check(self._lib.hsf_lb_advance(self._h, int(n_steps), p, where))

    def get_flow(self, rho=None, u=None):
        if rho is None:
            rho = np.empty(self.T)
        if u is None:
            u = np.empty(3 * self.T)
        pr, where = _ptr(rho, self.T)
        pu, _ = _ptr(u, 3 * self.T)
        self._check(self._lib.hsf_get_flow(self._h, pr, pu, where))
        return rho, u

    def cd_advance(self, mu, u=None):
        pm, where = _ptr(mu, self.nsp * self.T)
        pu, _ = _ptr(u, 3 * self.T)
        self._check(self._lib.hsf_cd_advance(self._h, pm, pu, where))

    def step(self, n_steps=1, tol=1e-8, max_iter=1000):
        st = (InvertStats * self.n_rep)()
        ev = ctypes.c_longlong(0)
        self._check(self._lib.hsf_step(self._h, int(n_steps), float(tol), int(max_iter), st, ctypes.byref(ev)))
        return [s.as_dict() for s in st], ev.value

    def get_state(self):
        """Checkpoint of the state a continuation reads (bytes)."""
        n = self._lib.hsf_state_size(self._h)
        buf = np.empty(n, dtype=np.uint8)
        self._check(self._lib.hsf_get_state(self._h, ctypes.c_void_p(buf.ctypes.data), n))
        return buf

    def set_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self._lib.hsf_set_state(self._h, ctypes.c_void_p(buf.ctypes.data), buf.size))

    def set_integrator(self, crank_nicolson=True, tol=1e-10, max_newton=20, krylov_dim=40):
        """Crank-Nicolson (implicit) or explicit diffusion in the coupled steps."""
        scheme = CD_CRANK_NICOLSON if crank_nicolson else CD_EXPLICIT
        self._check(self._lib.hsf_set_integrator(self._h, scheme, float(tol), int(max_newton), int(krylov_dim)))

    def cn_stats(self):
        st = CnStats()
        self._check(self._lib.hsf_get_cn_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def set_noise(self, cd=True, lb=True, omega=400.0, seed=0, step=0):
        """Thermal noise: composition noise (eq. 5) and/or LB mode noise (eq. 13)."""
        flags = (NOISE_CD if cd else 0) | (NOISE_LB if lb else 0)
        self._check(self._lib.hsf_set_noise(self._h, flags, float(omega), int(seed), int(step)))

    def noise_step(self):
        v = ctypes.c_ulonglong()
        self._check(self._lib.hsf_get_noise_step(self._h, ctypes.byref(v)))
        return int(v.value)

    def set_hydro(self, on):
        self._check(self._lib.hsf_set_hydro(self._h, int(bool(on))))

    def set_tile(self, cfg):
        arr = (ctypes.c_int * 4)(*[int(v) for v in cfg])
        self._check(self._lib.hsf_set_tile(self._h, arr))

    def get_tile(self):
        arr = (ctypes.c_int * 4)()
        self._check(self._lib.hsf_get_tile(self._h, arr))
        return tuple(arr[:])

    def autotune(self, reps=3):
        """Pick the fastest propagator tiling for this context; returns (cfg, ms per evaluation)."""
        ms = ctypes.c_double(0.0)
        self._check(self._lib.hsf_autotune(self._h, int(reps), ctypes.byref(ms)))
        return self.get_tile(), ms.value

    def set_solver(self, precond=False, refine=False):
        """Plain Fletcher-Reeves (default) or the diagonally preconditioned variant; refine:
        FP32 contexts finish inversions below a residual of 1e-5 with FP64 evaluations."""
        flags = (SOLVER_PRECOND if precond else 0) | (SOLVER_REFINE if refine else 0)
        self._check(self._lib.hsf_set_solver(self._h, flags))

    def get_work(self, reset=False):
        """(evaluations, sum over replicas of evaluations x sites) since the last reset."""
        ev = ctypes.c_longlong(0)
        se = ctypes.c_double(0.0)
        self._check(self._lib.hsf_get_work(self._h, ctypes.byref(ev), ctypes.byref(se), int(bool(reset))))
        return ev.value, se.value

    def set_warm(self, warm):
        """Warm start of hsf_step's inversions (WARM_CURRENT, WARM_LOCAL, WARM_EXTRAP, WARM_NET,
        WARM_NET_DELTA, WARM_NET_EXTRAP)."""
        self._check(self._lib.hsf_set_warm(self._h, int(warm)))

    def set_net_gate(self, min_iters):
        """Use the network only after inversions of at least min_iters iterations (0: always)."""
        self._check(self._lib.hsf_set_net_gate(self._h, int(min_iters)))

    def attach_net(self, net):
        self._check(self._lib.hsf_attach_net(self._h, net._h if net is not None else None))
        self._net = net   # keep it alive while attached

    def set_timing(self, on):
        self._check(self._lib.hsf_set_timing(self._h, int(bool(on))))

    def get_timing(self):
        """{kernel family: (total ms, launches)} since the last read."""
        ms = (ctypes.c_double * K_COUNT)()
        cnt = (ctypes.c_longlong * K_COUNT)()
        self._check(self._lib.hsf_get_timing(self._h, ms, cnt))
        return {KERNEL_NAMES[k]: (ms[k], cnt[k]) for k in range(K_COUNT)}

    def set_step_log(self, on=True):
        """Keep one record per replica and successful coupled step (hsf_set_step_log)."""
        self._check(self._lib.hsf_set_step_log(self._h, int(bool(on))))

    def read_step_log(self, max_records=4096):
        """The unread step records, oldest first, as dicts (hsf_read_step_log)."""
        out = []
        buf = (StepRecord * max_records)()
        while True:
            n = ctypes.c_int(0)
            self._check(self._lib.hsf_read_step_log(self._h, buf, int(max_records), ctypes.byref(n)))
            out.extend(buf[k].as_dict() for k in range(n.value))
            if n.value < max_records:
                return out

    def write_step_log(self, path):
        """Append the unread step records to a JSON-lines file; returns how many."""
        import json
        recs = self.read_step_log()
        with open(path, "a") as f:
            for r in recs:
                f.write(json.dumps(r) + "\n")
        return len(recs)


class Net:
    """The warm-start U-Net (FP32 boundary arrays [batch][channel][L][L][L]; L a
    multiple of 2^(depth - 1))."""

    def __init__(self, in_ch, out_ch=2, widths=(8, 16, 24, 32), seed=0, stream=None):
        """widths: 1 to 4 level widths (the number given is the depth of the U-Net)."""
        lib = load()
        widths = tuple(int(v) for v in widths)
        if not 1 <= len(widths) <= 4:
            raise ValueError("1 to 4 widths")
        w = (ctypes.c_int * 4)(*(widths + (0,) * (4 - len(widths))))
        h = ctypes.c_void_p()
        rc = lib.hsf_net_create(int(in_ch), int(out_ch), w, ctypes.c_ulonglong(seed), ctypes.byref(h))
        if rc != HSF_OK:
            raise HsfError(rc, "hsf_net_create failed")
        self._h, self._lib = h, lib
        self.in_ch, self.out_ch, self.widths = in_ch, out_ch, tuple(widths)
        self.n_params = lib.hsf_net_num_params(h)
        if stream is not None:
            raw = getattr(stream, "cuda_stream", stream)
            self._check(lib.hsf_net_set_stream(h, ctypes.c_void_p(raw or 0)))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hsf_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != HSF_OK:
            raise HsfError(rc, self._lib.hsf_net_last_error(self._h).decode())

    def set_params(self, p):
        ptr, where = _ptr32(p, self.n_params)
        self._check(self._lib.hsf_net_set_params(self._h, ptr, where))

    def set_input_norm(self, shift, scale):
        sh = (ctypes.c_float * self.in_ch)(*[float(v) for v in shift])
        sc = (ctypes.c_float * self.in_ch)(*[float(v) for v in scale])
        self._check(self._lib.hsf_net_set_input_norm(self._h, sh, sc))

    def set_output_scale(self, scale):
        sc = (ctypes.c_float * self.out_ch)(*[float(v) for v in scale])
        self._check(self._lib.hsf_net_set_output_scale(self._h, sc))

    def get_params(self):
        out = np.empty(self.n_params, dtype=np.float32)
        ptr, where = _ptr32(out, self.n_params)
        self._check(self._lib.hsf_net_get_params(self._h, ptr, where))
        return out

    def forward(self, x, batch, L, out=None):
        if out is None:
            out = np.empty(batch * self.out_ch * L ** 3, dtype=np.float32)
        pi, where = _ptr32(x, batch * self.in_ch * L ** 3)
        po, _ = _ptr32(out, batch * self.out_ch * L ** 3)
        self._check(self._lib.hsf_net_forward(self._h, pi, po, int(batch), int(L), where))
        return out

    def loss_grad(self, x, target, batch, L, with_grad=True):
        grad = np.empty(self.n_params, dtype=np.float32) if with_grad else None
        loss = ctypes.c_double(0.0)
        pi, where = _ptr32(x, batch * self.in_ch * L ** 3)
        pt, _ = _ptr32(target, batch * self.out_ch * L ** 3)
        pg, _ = _ptr32(grad, self.n_params)
        self._check(self._lib.hsf_net_loss_grad(self._h, pi, pt, int(batch), int(L), ctypes.byref(loss), pg, where))
        return loss.value, grad

    def train_step(self, x, target, batch, L, lr):
        loss = ctypes.c_double(0.0)
        pi, where = _ptr32(x, batch * self.in_ch * L ** 3)
        pt, _ = _ptr32(target, batch * self.out_ch * L ** 3)
        self._check(self._lib.hsf_net_train_step(self._h, pi, pt, int(batch), int(L), ctypes.c_float(lr),
                                                 ctypes.byref(loss), where))
        return loss.value

    def make_sample(self, phi, phi_n, phi_p, w, w_n, w_p, nsp, V, mode, x, y):
        """hsf_net_make_sample on device tensors (float64 states, float32 outputs)."""
        def p(t):
            return None if t is None else ctypes.c_void_p(t.data_ptr())
        self._check(self._lib.hsf_net_make_sample(self._h, p(phi), p(phi_n), p(phi_p), p(w), p(w_n), p(w_p),
                                                  int(nsp), int(V), int(mode), p(x), p(y)))

    def affine(self, x, batch, channels, V, shift, scale):
        """x_c = (x_c - shift[c]) * scale[c] on a float32 device tensor [batch][channels][V]."""
        sh = (ctypes.c_float * channels)(*[float(v) for v in shift])
        sc = (ctypes.c_float * channels)(*[float(v) for v in scale])
        self._check(self._lib.hsf_net_affine(self._h, ctypes.c_void_p(x.data_ptr()), int(batch), int(channels),
                                             int(V), sh, sc))

    def channel_moments(self, x, batch, channels, V):
        """Per-channel (mean, rms) of a float32 device tensor [batch][channels][V]."""
        mean = (ctypes.c_double * channels)()
        rms = (ctypes.c_double * channels)()
        self._check(self._lib.hsf_net_channel_moments(self._h, ctypes.c_void_p(x.data_ptr()), int(batch),
                                                      int(channels), int(V), mean, rms))
        return list(mean), list(rms)
