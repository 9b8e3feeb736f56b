"""Thin ctypes binding of libsdpd (include/sdpd.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies device memory (float64 / int32 CUDA tensors on ROCm) and the
stream.  The binding refuses to run without the compiled library.
"""
import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsdpd.so")

OK, EINVAL, EHIP, ENOMEM, ECELLCAP, ENEGEPS, ENONFINITE, ECAPACITY = 0, -1, -2, -3, -4, -5, -6, -7
KERNEL_LUCY, KERNEL_CUBIC = 0, 1
FD_EMS, FD_AMS, FD_SSA, FD_NONE = 0, 1, 2, 3
FP64, MIXED = 0, 1
SWEEP_AUTO, SWEEP_ONE, SWEEP_PER_GROUP = 0, 1, 2
BATCH_AUTO, BATCH_FUSED, BATCH_GRAPHS, BATCH_FUSED_FLOW = 0, 1, 2, 3
TIMING_CLASSES = ("cells", "density", "fd", "forces", "observe", "schedule")

EXPORTS = ("sdpd_create", "sdpd_destroy", "sdpd_build_cells", "sdpd_cell_info",
           "sdpd_copy_cell_start", "sdpd_density",
           "sdpd_forces", "sdpd_fd_metropolis", "sdpd_step", "sdpd_observe", "sdpd_sync",
           "sdpd_set_timing", "sdpd_timing", "sdpd_tune", "sdpd_get_tuning",
           "sdpd_fd_schedule_size", "sdpd_set_sweep_mode", "sdpd_sweep_mode", "sdpd_autotune",
           "sdpd_set_timing_mask",
           "sdpd_batch_create", "sdpd_batch_create_layout", "sdpd_batch_layout",
           "sdpd_batch_run", "sdpd_batch_destroy", "sdpd_adjoint_forward", "sdpd_adjoint_backward",
           "sdpd_adjoint_vjp", "sdpd_observe_noalloc", "sdpd_strerror",
           "sdpd_abi_version")


class _Params(C.Structure):
    _fields_ = [("n", C.c_int64), ("box", C.c_double * 3),
                ("m", C.c_double), ("h", C.c_double), ("kB", C.c_double),
                ("Cv", C.c_double), ("A", C.c_double), ("rho0", C.c_double),
                ("eta", C.c_double), ("zeta", C.c_double), ("dt", C.c_double),
                ("fd_every", C.c_int32), ("kernel", C.c_int32), ("fd", C.c_int32),
                ("prec", C.c_int32), ("seed", C.c_uint64), ("replica", C.c_uint32),
                ("cell_cap", C.c_int32), ("ncell", C.c_int32 * 3)]


class _State(C.Structure):
    _fields_ = [("q", C.c_void_p), ("p", C.c_void_p), ("eps", C.c_void_p),
                ("rho", C.c_void_p), ("f", C.c_void_p), ("id", C.c_void_p)]


class _Tuning(C.Structure):
    _fields_ = [("fd_tasks", C.c_int32 * 4), ("fd_lds_particles", C.c_int32 * 4),
                ("fd_lds_pairs", C.c_int32 * 4)]


class _Stats(C.Structure):
    _fields_ = [("proposed", C.c_uint64), ("rej_energy", C.c_uint64),
                ("rej_ratio", C.c_uint64), ("marginal", C.c_uint64), ("negeps", C.c_uint64),
                ("E", C.c_double), ("Eint", C.c_double), ("KE", C.c_double),
                ("P", C.c_double * 3), ("min_eps", C.c_double)]


class _Cotangent(C.Structure):
    _fields_ = [("dq", C.c_void_p), ("dp", C.c_void_p), ("deps", C.c_void_p),
                ("drho", C.c_void_p)]


class _Gradient(C.Structure):
    _fields_ = [("dq0", C.c_void_p), ("dp0", C.c_void_p), ("deps0", C.c_void_p),
                ("dA", C.c_double), ("dCv", C.c_double), ("drho0", C.c_double)]


def _stats(s: _Stats) -> dict:
    return {"proposed": s.proposed, "rej_energy": s.rej_energy, "rej_ratio": s.rej_ratio,
            "marginal": s.marginal, "negeps": s.negeps, "E": s.E, "Eint": s.Eint, "KE": s.KE,
            "P": tuple(s.P), "min_eps": s.min_eps}


_lib = None


def lib():
    """Load libsdpd.so; fail loudly if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__; __graft_entry__.build()'`")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded (one runtime per process; loading the library first made
        # torch and the library disagree about the device)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64 = C.c_void_p, C.c_int, C.c_int64, C.c_uint64
        SP = C.POINTER(_State)
        sig = {
            "sdpd_create": [C.POINTER(_Params), vp, C.POINTER(vp)],
            "sdpd_destroy": [vp],
            "sdpd_build_cells": [vp, SP],
            "sdpd_cell_info": [vp, C.POINTER(C.c_int32), C.POINTER(vp)],
            "sdpd_copy_cell_start": [vp, vp, i64],
            "sdpd_density": [vp, SP, i32],
            "sdpd_forces": [vp, SP],
            "sdpd_fd_metropolis": [vp, SP, u64, C.POINTER(_Stats)],
            "sdpd_step": [vp, SP, u64, i32, C.POINTER(_Stats)],
            "sdpd_observe": [vp, SP, C.POINTER(_Stats)],
            "sdpd_sync": [vp],
            "sdpd_set_timing": [vp, i32],
            "sdpd_set_timing_mask": [vp, C.c_uint32],
            "sdpd_timing": [vp, C.POINTER(C.c_double), C.POINTER(i64)],
            "sdpd_tune": [vp, C.POINTER(_Tuning)],
            "sdpd_autotune": [vp, SP, i32, C.POINTER(_Tuning)],
            "sdpd_get_tuning": [vp, C.POINTER(_Tuning)],
            "sdpd_fd_schedule_size": [vp, C.POINTER(i64), C.POINTER(i64)],
            "sdpd_batch_create": [C.POINTER(vp), C.POINTER(_State), i32, C.POINTER(vp)],
            "sdpd_batch_create_layout": [C.POINTER(vp), C.POINTER(_State), i32, i32, i32,
                                         C.POINTER(vp)],
            "sdpd_batch_layout": [vp],
            "sdpd_batch_run": [vp, u64, i32],
            "sdpd_batch_destroy": [vp],
            "sdpd_adjoint_forward": [vp, SP, i32, i32],
            "sdpd_adjoint_backward": [vp, vp, vp, vp, vp, vp, C.POINTER(C.c_double)],
            "sdpd_adjoint_vjp": [vp, C.POINTER(_Cotangent), C.POINTER(_Gradient)],
            "sdpd_observe_noalloc": [C.POINTER(_Params), SP, vp, vp],
            "sdpd_abi_version": [],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.sdpd_strerror.argtypes = [C.c_int]
        L.sdpd_strerror.restype = C.c_char_p
        _lib = L
    return _lib


class SdpdError(RuntimeError):
    def __init__(self, rc: int, what: str):
        msg = lib().sdpd_strerror(rc).decode()
        super().__init__(f"{what}: {msg} ({rc})")
        self.rc = rc


def _check(rc: int, what: str):
    if rc != OK:
        raise SdpdError(rc, what)


@dataclass
class SdpdParams:
    n: int
    box: tuple
    m: float = 1.0
    h: float = 2.5
    kB: float = 1.0
    Cv: float = 10.0
    A: float = 0.0           # 0: the library's default Cv / (3 kB)
    rho0: float = 1.0
    eta: float = 1.0
    zeta: float = 0.0
    dt: float = 0.005
    fd_every: int = 1
    kernel: int = KERNEL_LUCY
    fd: int = FD_EMS
    prec: int = 0
    seed: int = 0
    replica: int = 0
    cell_cap: int = 64
    ncell: tuple = (0, 0, 0)

    def c(self) -> _Params:
        box = tuple(self.box) if np.ndim(self.box) else (float(self.box),) * 3
        return _Params(int(self.n), (C.c_double * 3)(*box), self.m, self.h, self.kB, self.Cv,
                       0.0 if self.A is None else float(self.A),
                       self.rho0, self.eta, self.zeta, self.dt, int(self.fd_every),
                       int(self.kernel), int(self.fd), int(self.prec), int(self.seed),
                       int(self.replica), int(self.cell_cap), (C.c_int32 * 3)(*self.ncell))


class DeviceState:
    """State in device memory: float64 (3, n) q, p, f; (n,) eps, rho; int32 ids."""

    def __init__(self, q, p, eps, rho, f, ids):
        self.q, self.p, self.eps, self.rho, self.f, self.id = q, p, eps, rho, f, ids

    @staticmethod
    def from_numpy(q, p, eps, ids, rho=None, f=None, device="cuda"):
        import torch
        n = eps.shape[0]
        t = lambda a, shape: torch.as_tensor(np.ascontiguousarray(a, np.float64).reshape(shape),
                                             device=device).contiguous()
        return DeviceState(t(q, (3, n)), t(p, (3, n)), t(eps, (n,)),
                           t(np.zeros(n) if rho is None else rho, (n,)),
                           t(np.zeros((3, n)) if f is None else f, (3, n)),
                           torch.as_tensor(np.ascontiguousarray(ids).astype(np.int32),
                                           device=device).contiguous())

    def to_numpy(self) -> dict:
        return {"q": self.q.cpu().numpy(), "p": self.p.cpu().numpy(),
                "eps": self.eps.cpu().numpy(), "rho": self.rho.cpu().numpy(),
                "f": self.f.cpu().numpy(), "id": self.id.cpu().numpy().astype(np.uint32)}

    def c(self) -> _State:
        for t in (self.q, self.p, self.eps, self.rho, self.f, self.id):
            if not (t.is_cuda and t.is_contiguous()):
                raise ValueError("state tensors must be contiguous device tensors")
        return _State(self.q.data_ptr(), self.p.data_ptr(), self.eps.data_ptr(),
                      self.rho.data_ptr(), self.f.data_ptr(), self.id.data_ptr())


def observe_noalloc(params: SdpdParams, s: DeviceState, out, stream=None):
    """sdpd_observe_noalloc: E, Eint, KE, P (3), min eps of s into the float64
    device tensor out (7 elements), on stream (default: torch's current)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
            and out.numel() >= 7):
        raise ValueError("out must be a contiguous float64 device tensor of 7 elements")
    _check(lib().sdpd_observe_noalloc(C.byref(params.c()), C.byref(s.c()),
                                      C.c_void_p(stream.cuda_stream), C.c_void_p(out.data_ptr())),
           "sdpd_observe_noalloc")


class Context:
    """An sdpd_ctx bound to one stream (default: torch's current stream)."""

    def __init__(self, params: SdpdParams, stream=None):
        import torch
        self.params = params
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        _check(lib().sdpd_create(C.byref(params.c()), C.c_void_p(stream.cuda_stream),
                                 C.byref(h)), "sdpd_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().sdpd_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def build_cells(self, s: DeviceState):
        _check(lib().sdpd_build_cells(self._h, C.byref(s.c())), "sdpd_build_cells")

    def cell_info(self):
        """(ncell tuple, device pointer of cell_start)."""
        nc = (C.c_int32 * 3)()
        ptr = C.c_void_p()
        _check(lib().sdpd_cell_info(self._h, nc, C.byref(ptr)), "sdpd_cell_info")
        return tuple(nc), ptr.value

    def cell_start(self):
        """Copy of cell_start (ncell + 1 uint32) on the host (synchronises)."""
        nc, _ = self.cell_info()
        out = np.zeros(nc[0] * nc[1] * nc[2] + 1, np.uint32)
        _check(lib().sdpd_copy_cell_start(self._h, out.ctypes.data_as(C.c_void_p), out.size),
               "sdpd_copy_cell_start")
        return out

    def density(self, s: DeviceState, update_eps: bool = False):
        _check(lib().sdpd_density(self._h, C.byref(s.c()), int(bool(update_eps))), "sdpd_density")

    def forces(self, s: DeviceState):
        _check(lib().sdpd_forces(self._h, C.byref(s.c())), "sdpd_forces")

    def fd_metropolis(self, s: DeviceState, step: int, stats: bool = True):
        st = _Stats()
        _check(lib().sdpd_fd_metropolis(self._h, C.byref(s.c()), int(step),
                                        C.byref(st) if stats else None), "sdpd_fd_metropolis")
        return _stats(st) if stats else None

    def step(self, s: DeviceState, step0: int, nsteps: int, stats: bool = True):
        arr = (_Stats * max(nsteps, 1))()
        _check(lib().sdpd_step(self._h, C.byref(s.c()), int(step0), int(nsteps),
                               arr if stats else None), "sdpd_step")
        return [_stats(arr[k]) for k in range(nsteps)] if stats else None

    def observe(self, s: DeviceState):
        st = _Stats()
        _check(lib().sdpd_observe(self._h, C.byref(s.c()), C.byref(st)), "sdpd_observe")
        return _stats(st)

    def sync(self):
        _check(lib().sdpd_sync(self._h), "sdpd_sync")

    def set_timing(self, enable: bool):
        _check(lib().sdpd_set_timing(self._h, int(bool(enable))), "sdpd_set_timing")

    def set_timing_classes(self, classes):
        """Time only the named classes (names of TIMING_CLASSES)."""
        mask = 0
        for k in classes:
            mask |= 1 << TIMING_CLASSES.index(k)
        _check(lib().sdpd_set_timing_mask(self._h, C.c_uint32(mask)), "sdpd_set_timing_mask")

    def timing(self) -> dict:
        ms = (C.c_double * len(TIMING_CLASSES))()
        cnt = (C.c_int64 * len(TIMING_CLASSES))()
        _check(lib().sdpd_timing(self._h, ms, cnt), "sdpd_timing")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(TIMING_CLASSES)}

    def tune(self, fd_tasks=None, lds_particles=None, lds_pairs=None):
        """F/D execution tuning per phase class (own cell, face, edge, corner):
        tasks per workgroup and the LDS capacity of a workgroup; None or 0
        keeps the current value."""
        t = _Tuning()
        for field, vals in (("fd_tasks", fd_tasks), ("fd_lds_particles", lds_particles),
                            ("fd_lds_pairs", lds_pairs)):
            arr = getattr(t, field)
            for k, v in enumerate(vals or (0, 0, 0, 0)):
                arr[k] = int(v)
        _check(lib().sdpd_tune(self._h, C.byref(t)), "sdpd_tune")

    def autotune(self, s: "DeviceState", trials: int = 3) -> dict:
        """Time candidate F/D tunings on scratch copies of s's momenta and
        energies and keep the fastest (cells and masks must be current);
        returns the tuning in use."""
        t = _Tuning()
        _check(lib().sdpd_autotune(self._h, C.byref(s.c()), int(trials), C.byref(t)),
               "sdpd_autotune")
        return {"fd_tasks": tuple(t.fd_tasks), "lds_particles": tuple(t.fd_lds_particles),
                "lds_pairs": tuple(t.fd_lds_pairs)}

    def adjoint_forward(self, s: DeviceState, nsteps: int, checkpoint_every: int = 10):
        _check(lib().sdpd_adjoint_forward(self._h, C.byref(s.c()), int(nsteps),
                                          int(checkpoint_every)), "sdpd_adjoint_forward")

    def adjoint_backward(self, dJ_dq, dJ_dp):
        """dJ/dq_K, dJ/dp_K: float64 (3, n) device tensors indexed by particle
        id.  Returns (dJ/dq0, dJ/dp0, dJ/deps0, dJ/dA), id-indexed tensors."""
        import torch
        n = dJ_dq.shape[1]
        dq0 = torch.empty((3, n), dtype=torch.float64, device=dJ_dq.device)
        dp0 = torch.empty_like(dq0)
        de0 = torch.empty((n,), dtype=torch.float64, device=dJ_dq.device)
        dA = C.c_double()
        a, b = dJ_dq.contiguous(), dJ_dp.contiguous()
        _check(lib().sdpd_adjoint_backward(self._h, a.data_ptr(), b.data_ptr(), dq0.data_ptr(),
                                           dp0.data_ptr(), de0.data_ptr(), C.byref(dA)),
               "sdpd_adjoint_backward")
        return dq0, dp0, de0, dA.value

    def adjoint_vjp(self, dq, dp, deps=None, drho=None):
        """Reverse pass from the cotangents of the final state, all float64
        device tensors indexed by particle id: dq, dp (3, n) and optionally
        deps, drho (n,).  Returns a dict with dq0, dp0 (3, n), deps0 (n,)
        tensors and the scalars dA, dCv (at fixed A) and drho0."""
        import torch
        n = dq.shape[1]
        out = {"dq0": torch.empty((3, n), dtype=torch.float64, device=dq.device),
               "dp0": torch.empty((3, n), dtype=torch.float64, device=dq.device),
               "deps0": torch.empty((n,), dtype=torch.float64, device=dq.device)}
        keep = [t.contiguous() if t is not None else None for t in (dq, dp, deps, drho)]
        ptr = lambda t: None if t is None else t.data_ptr()
        ct = _Cotangent(*[ptr(t) for t in keep])
        gr = _Gradient(out["dq0"].data_ptr(), out["dp0"].data_ptr(), out["deps0"].data_ptr(),
                       0.0, 0.0, 0.0)
        _check(lib().sdpd_adjoint_vjp(self._h, C.byref(ct), C.byref(gr)), "sdpd_adjoint_vjp")
        out.update(dA=gr.dA, dCv=gr.dCv, drho0=gr.drho0)
        return out

    def fd_schedule_size(self):
        """(active pairs, staged particle entries) of the last F/D sweep."""
        a, b = C.c_int64(), C.c_int64()
        _check(lib().sdpd_fd_schedule_size(self._h, C.byref(a), C.byref(b)),
               "sdpd_fd_schedule_size")
        return a.value, b.value

    def get_tuning(self) -> dict:
        t = _Tuning()
        _check(lib().sdpd_get_tuning(self._h, C.byref(t)), "sdpd_get_tuning")
        return {"fd_tasks": tuple(t.fd_tasks), "lds_particles": tuple(t.fd_lds_particles),
                "lds_pairs": tuple(t.fd_lds_pairs)}

    def set_sweep_mode(self, mode: int):
        """SWEEP_AUTO, SWEEP_ONE or SWEEP_PER_GROUP (results are identical)."""
        _check(lib().sdpd_set_sweep_mode(self._h, int(mode)), "sdpd_set_sweep_mode")

    def sweep_mode(self) -> tuple:
        """(mode set, layout in use)."""
        u = C.c_int(0)
        m = lib().sdpd_sweep_mode(self._h, C.byref(u))
        if m < 0:
            _check(m, "sdpd_sweep_mode")
        return m, u.value

    def prepare(self, s: DeviceState):
        """cells, density without energy update, forces: the entry state of step()."""
        self.build_cells(s)
        self.density(s, update_eps=False)
        self.forces(s)


class Batch:
    """Many boxes (contexts with their states) advanced together: by default
    every stage of a step is one launch for all boxes (BATCH_FUSED; with
    BATCH_FUSED_FLOW the F/D sweeps of all boxes are one persistent launch);
    with BATCH_GRAPHS each box's own launches are captured."""

    def __init__(self, contexts, states, layout=BATCH_AUTO, parts=0):
        self._ctx = list(contexts)
        self._st = list(states)
        n = len(self._ctx)
        handles = (C.c_void_p * n)(*[c._h.value for c in self._ctx])
        self._cst = (_State * n)(*[s.c() for s in self._st])
        self._h = C.c_void_p()
        _check(lib().sdpd_batch_create_layout(handles, self._cst, n, int(layout), int(parts),
                                              C.byref(self._h)), "sdpd_batch_create_layout")

    def layout(self) -> int:
        """The layout in use (BATCH_FUSED, BATCH_FUSED_FLOW or BATCH_GRAPHS)."""
        m = lib().sdpd_batch_layout(self._h)
        if m < 0:
            _check(m, "sdpd_batch_layout")
        return m

    def run(self, step0: int, nsteps: int):
        _check(lib().sdpd_batch_run(self._h, int(step0), int(nsteps)), "sdpd_batch_run")

    def close(self):
        if self._h is not None and self._h.value:
            lib().sdpd_batch_destroy(self._h)
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
