"""ctypes wrapper of the C oracle (oracle/sdpd_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark.  The GPU library never imports or links this.
All arrays are numpy float64 / uint32, structure of arrays ((3, n) for
3-vectors), C-contiguous; functions work in place where the C does.
"""
import ctypes as C
from dataclasses import dataclass, field

import numpy as np

from .build import ensure_oracle, ensure_oracle_omp

KERNEL_LUCY, KERNEL_CUBIC = 0, 1
FD_EMS, FD_AMS, FD_SSA, FD_NONE = 0, 1, 2, 3
OK, EINVAL, ENOMEM, ECELLCAP, ENEGEPS, ENONFINITE = 0, -1, -3, -4, -5, -6


class _Params(C.Structure):
    _fields_ = [("n", C.c_int64), ("box", C.c_double * 3),
                ("m", C.c_double), ("h", C.c_double), ("kB", C.c_double),
                ("Cv", C.c_double), ("A", C.c_double), ("rho0", C.c_double),
                ("eta", C.c_double), ("zeta", C.c_double), ("dt", C.c_double),
                ("fd_every", C.c_int32), ("kernel", C.c_int32), ("fd_mode", C.c_int32),
                ("seed", C.c_uint64), ("replica", C.c_uint32), ("cell_cap", C.c_int32),
                ("ncell", C.c_int32 * 3)]


class _Stats(C.Structure):
    _fields_ = [("proposed", C.c_uint64), ("rej_energy", C.c_uint64),
                ("rej_ratio", C.c_uint64), ("marginal", C.c_uint64), ("negeps", C.c_uint64),
                ("E", C.c_double), ("Eint", C.c_double), ("KE", C.c_double),
                ("P", C.c_double * 3), ("min_eps", C.c_double)]


PAIRREC_DTYPE = np.dtype([("phase", np.int32), ("round", np.int32), ("i", np.int32),
                          ("j", np.int32), ("decision", np.int32), ("pad", np.int32),
                          ("a_minus_lnU", np.float64), ("bound_gap", np.float64)])


@dataclass
class OracleParams:
    n: int
    box: tuple
    m: float = 1.0
    h: float = 2.5
    kB: float = 1.0
    Cv: float = 10.0
    A: float = None          # default Cv / (3 kB)
    rho0: float = 1.0
    eta: float = 1.0
    zeta: float = 0.0
    dt: float = 0.005
    fd_every: int = 1
    kernel: int = KERNEL_LUCY
    fd_mode: int = FD_EMS
    seed: int = 0
    replica: int = 0
    cell_cap: int = 64
    ncell: tuple = (0, 0, 0)

    def c(self) -> _Params:
        A = self.A if self.A is not None else self.Cv / (3.0 * self.kB)
        box = self.box if np.ndim(self.box) else (self.box,) * 3
        return _Params(int(self.n), (C.c_double * 3)(*box), self.m, self.h, self.kB,
                       self.Cv, A, self.rho0, self.eta, self.zeta, self.dt,
                       int(self.fd_every), int(self.kernel), int(self.fd_mode),
                       int(self.seed), int(self.replica), int(self.cell_cap),
                       (C.c_int32 * 3)(*self.ncell))


def stats_dict(s: _Stats) -> dict:
    return {"proposed": s.proposed, "rej_energy": s.rej_energy, "rej_ratio": s.rej_ratio,
            "marginal": s.marginal, "negeps": s.negeps, "E": s.E, "Eint": s.Eint,
            "KE": s.KE, "P": tuple(s.P), "min_eps": s.min_eps}


_lib = None
_lib_omp = None
_D = C.POINTER(C.c_double)
_U32 = C.POINTER(C.c_uint32)


def lib_omp():
    """The OpenMP build of the same source (its so_step_parallel runs on
    several threads)."""
    global _lib_omp
    if _lib_omp is None:
        _lib_omp = _load(ensure_oracle_omp())
    return _lib_omp


def lib():
    global _lib
    if _lib is None:
        _lib = _load(ensure_oracle())
    return _lib


def _load(path):
    L = C.CDLL(path)
    PP, SP = C.POINTER(_Params), C.POINTER(_Stats)
    sig = {
        "so_kernel_w": (C.c_double, [C.c_int, C.c_double, C.c_double]),
        "so_kernel_f": (C.c_double, [C.c_int, C.c_double, C.c_double]),
        "so_entropy": (C.c_double, [PP, C.c_double, C.c_double]),
        "so_temperature": (C.c_double, [PP, C.c_double, C.c_double]),
        "so_pressure": (C.c_double, [PP, C.c_double, C.c_double]),
        "so_heat_capacity": (C.c_double, [PP, C.c_double, C.c_double]),
        "so_eps_at_entropy": (C.c_double, [PP, C.c_double, C.c_double]),
        "so_grid": (C.c_int, [PP, C.POINTER(C.c_int32)]),
        "so_build_cells": (C.c_int, [PP, _D, _D, _D, _D, _D, _U32, _U32]),
        "so_density": (C.c_int, [PP, _D, _U32, _D]),
        "so_density_bruteforce": (C.c_int, [PP, _D, _D]),
        "so_update_eps_const_entropy": (C.c_int, [PP, _D, _D, _D]),
        "so_forces": (C.c_int, [PP, _D, _D, _D, _U32, _D]),
        "so_forces_bruteforce": (C.c_int, [PP, _D, _D, _D, _D]),
        "so_philox4x32_10": (None, [_U32, _U32, _U32]),
        "so_pair_draws": (None, [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32,
                                 C.c_uint32, _D, _D]),
        "so_fd_coefficients": (None, [PP, C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_double, C.c_double, _D, _D]),
        "so_fd_log_ratio": (C.c_double, [PP, C.c_double, C.c_double, C.c_double,
                                         C.c_double, C.c_double, _D, _D, _D, C.c_double,
                                         _D, _D]),
        "so_fd_pair_list": (C.c_int, [PP, _D, _U32, C.c_void_p, C.c_int64,
                                      C.POINTER(C.c_int64)]),
        "so_fd_sweep": (C.c_int, [PP, _D, _D, _D, _D, _U32, _U32, C.c_uint64,
                                  C.c_double, SP, C.c_void_p, C.c_int64]),
        "so_fd_sweep_flip": (C.c_int, [PP, _D, _D, _D, _D, _U32, _U32, C.c_uint64,
                                       C.c_double, SP, C.c_void_p, C.c_int64,
                                       C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                       C.c_int64]),
        "so_observe": (C.c_int, [PP, _D, _D, SP]),
        "so_kick": (C.c_int, [PP, _D, _D, C.c_double]),
        "so_drift": (C.c_int, [PP, _D, _D, C.c_double]),
        "so_step": (C.c_int, [PP, _D, _D, _D, _D, _D, _U32, _U32, C.c_uint64,
                              C.c_int, SP]),
        "so_step_parallel": (C.c_int, [PP, _D, _D, _D, _D, _D, _U32, _U32, C.c_uint64,
                                       C.c_int, SP]),
        "so_threads": (C.c_int, [C.c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _u(a):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(_U32)


class OracleError(RuntimeError):
    def __init__(self, rc, what):
        super().__init__(f"oracle {what} returned {rc}")
        self.rc = rc


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


# ---------------------------------------------------------------- closure
def kernel_w(kernel, h, r):
    return lib().so_kernel_w(kernel, h, r)


def kernel_f(kernel, h, r):
    return lib().so_kernel_f(kernel, h, r)


def entropy(P, eps, rho):
    return lib().so_entropy(C.byref(P.c()), eps, rho)


def temperature(P, eps, rho):
    return lib().so_temperature(C.byref(P.c()), eps, rho)


def pressure(P, eps, rho):
    return lib().so_pressure(C.byref(P.c()), eps, rho)


def heat_capacity(P, eps, rho):
    return lib().so_heat_capacity(C.byref(P.c()), eps, rho)


def eps_at_entropy(P, S, rho):
    return lib().so_eps_at_entropy(C.byref(P.c()), S, rho)


def grid(P):
    nc = (C.c_int32 * 3)()
    _check(lib().so_grid(C.byref(P.c()), nc), "grid")
    return tuple(nc)


# ---------------------------------------------------------------- state ops
@dataclass
class State:
    """Host state, structure of arrays."""
    q: np.ndarray
    p: np.ndarray
    eps: np.ndarray
    rho: np.ndarray
    f: np.ndarray
    id: np.ndarray
    cell_start: np.ndarray = field(default=None)

    @staticmethod
    def from_arrays(q, p, eps, id, rho=None, f=None):
        n = eps.shape[0]
        return State(np.ascontiguousarray(q, np.float64).copy(),
                     np.ascontiguousarray(p, np.float64).copy(),
                     np.ascontiguousarray(eps, np.float64).copy(),
                     np.zeros(n) if rho is None else np.ascontiguousarray(rho, np.float64).copy(),
                     np.zeros((3, n)) if f is None else np.ascontiguousarray(f, np.float64).copy(),
                     np.ascontiguousarray(id, np.uint32).copy())

    def copy(self):
        return State(self.q.copy(), self.p.copy(), self.eps.copy(), self.rho.copy(),
                     self.f.copy(), self.id.copy(),
                     None if self.cell_start is None else self.cell_start.copy())


def build_cells(P, S: State):
    nc = grid(P)
    S.cell_start = np.zeros(nc[0] * nc[1] * nc[2] + 1, np.uint32)
    rc = lib().so_build_cells(C.byref(P.c()), _d(S.q), _d(S.p), _d(S.eps), _d(S.rho),
                              _d(S.f), _u(S.id), _u(S.cell_start))
    _check(rc, "build_cells")
    return S.cell_start


def density(P, S: State):
    out = np.empty(P.n)
    _check(lib().so_density(C.byref(P.c()), _d(S.q), _u(S.cell_start), _d(out)), "density")
    return out


def density_bruteforce(P, q):
    out = np.empty(P.n)
    _check(lib().so_density_bruteforce(C.byref(P.c()), _d(np.ascontiguousarray(q)), _d(out)),
           "density_bruteforce")
    return out


def update_eps_const_entropy(P, eps, rho_old, rho_new):
    _check(lib().so_update_eps_const_entropy(C.byref(P.c()), _d(eps), _d(rho_old),
                                             _d(rho_new)), "update_eps")
    return eps


def forces(P, S: State):
    out = np.empty((3, P.n))
    _check(lib().so_forces(C.byref(P.c()), _d(S.q), _d(S.rho), _d(S.eps),
                           _u(S.cell_start), _d(out)), "forces")
    return out


def forces_bruteforce(P, q, rho, eps):
    out = np.empty((3, P.n))
    _check(lib().so_forces_bruteforce(C.byref(P.c()), _d(np.ascontiguousarray(q)),
                                      _d(np.ascontiguousarray(rho)),
                                      _d(np.ascontiguousarray(eps)), _d(out)),
           "forces_bruteforce")
    return out


def prepare(P, S: State):
    """cells, density (no energy update) and forces for a fresh state."""
    build_cells(P, S)
    S.rho[:] = density(P, S)
    S.f[:] = forces(P, S)
    return S


# ---------------------------------------------------------------- random numbers
def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().so_philox4x32_10(_u(c), _u(k), _u(out))
    return out


def pair_draws(seed, step, id_i, id_j, replica=0):
    G = np.zeros(3)
    U = C.c_double()
    lib().so_pair_draws(seed, step, id_i, id_j, replica, _d(G), C.byref(U))
    return G, U.value


# ---------------------------------------------------------------- F/D
def fd_coefficients(P, F, rho_i, rho_j, eps_i, eps_j, dt):
    a = np.zeros(2)
    z = np.zeros(2)
    lib().so_fd_coefficients(C.byref(P.c()), F, rho_i, rho_j, eps_i, eps_j, dt, _d(a), _d(z))
    return a, z


def fd_log_ratio(P, F, rho_i, rho_j, eps_i, eps_j, v, e, G, dt):
    v = np.ascontiguousarray(v, np.float64)
    e = np.ascontiguousarray(e, np.float64)
    G = np.ascontiguousarray(G, np.float64)
    vnew = np.zeros(3)
    en = np.zeros(2)
    a = lib().so_fd_log_ratio(C.byref(P.c()), F, rho_i, rho_j, eps_i, eps_j, _d(v), _d(e),
                              _d(G), dt, _d(vnew), _d(en))
    return a, vnew, en


def fd_pair_list(P, S: State):
    cnt = C.c_int64()
    lib().so_fd_pair_list(C.byref(P.c()), _d(S.q), _u(S.cell_start), None, 0, C.byref(cnt))
    out = np.zeros(cnt.value, PAIRREC_DTYPE)
    _check(lib().so_fd_pair_list(C.byref(P.c()), _d(S.q), _u(S.cell_start),
                                 out.ctypes.data_as(C.c_void_p), cnt.value, C.byref(cnt)),
           "fd_pair_list")
    return out


def fd_sweep(P, S: State, step, dt_fd=None, log=False, flip=()):
    """One F/D sweep in place.  Returns (rc, stats, pair log or None).
    flip: {position in sweep order: kind}, kind bit 0 inverts the outcome of
    the energy bound and bit 1 that of the Metropolis test of that pair (a
    test control for decisions inside the rounding margin)."""
    st = _Stats()
    rec = None
    cap = 0
    if log:
        cap = len(fd_pair_list(P, S))
        rec = np.zeros(cap, PAIRREC_DTYPE)
    dt = P.dt * P.fd_every if dt_fd is None else dt_fd
    out = None if rec is None else rec.ctypes.data_as(C.c_void_p)
    if len(flip):
        pos = sorted(int(k) for k in flip)
        fl = np.ascontiguousarray(pos, np.int64)
        kind = np.ascontiguousarray([int(flip[k]) for k in pos], np.int32)
        rc = lib().so_fd_sweep_flip(C.byref(P.c()), _d(S.q), _d(S.p), _d(S.eps), _d(S.rho),
                                    _u(S.id), _u(S.cell_start), step, dt, C.byref(st), out,
                                    cap, fl.ctypes.data_as(C.POINTER(C.c_int64)),
                                    kind.ctypes.data_as(C.POINTER(C.c_int32)), len(fl))
    else:
        rc = lib().so_fd_sweep(C.byref(P.c()), _d(S.q), _d(S.p), _d(S.eps), _d(S.rho),
                               _u(S.id), _u(S.cell_start), step, dt, C.byref(st), out, cap)
    return rc, stats_dict(st), rec


def observe(P, S: State):
    st = _Stats()
    lib().so_observe(C.byref(P.c()), _d(S.p), _d(S.eps), C.byref(st))
    return stats_dict(st)


def kick(P, S: State, half_dt):
    lib().so_kick(C.byref(P.c()), _d(S.p), _d(S.f), half_dt)


def drift(P, S: State, dt):
    lib().so_drift(C.byref(P.c()), _d(S.q), _d(S.p), dt)


def step(P, S: State, step0, nsteps):
    """nsteps full steps in place; returns (rc, list of per-step stats)."""
    return _step(lib().so_step, P, S, step0, nsteps)


def step_parallel(P, S: State, step0, nsteps, threads=0, omp=True):
    """The parallel variant of step (the same result bit for bit): on
    `threads` OpenMP threads (0 = the runtime's default) with the OpenMP
    build, or on one thread with the plain build (omp=False).  Returns
    (rc, per-step stats, threads used)."""
    L = lib_omp() if omp else lib()
    used = L.so_threads(int(threads))
    rc, st = _step(L.so_step_parallel, P, S, step0, nsteps)
    return rc, st, used


def _step(fn, P, S, step0, nsteps):
    if S.cell_start is None:
        nc = grid(P)
        S.cell_start = np.zeros(nc[0] * nc[1] * nc[2] + 1, np.uint32)
    st = (_Stats * max(nsteps, 1))()
    rc = fn(C.byref(P.c()), _d(S.q), _d(S.p), _d(S.eps), _d(S.rho), _d(S.f), _u(S.id),
            _u(S.cell_start), step0, nsteps, st)
    return rc, [stats_dict(st[k]) for k in range(nsteps)]
