"""ctypes binding of libnpweno.so (the C ABI of include/npweno.h).

Argument marshalling only: every step of the scheme runs in the library's HIP kernels.  Arrays
may be numpy arrays (host) or torch CUDA tensors (device, passed by data_ptr()); the stream is
torch's current stream unless one is given.  Loading fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnpweno.so")

NPW_ABI_VERSION = 2
OK, EINVAL, ENOMEM, EHIP, ENONFINITE, ENONPHYSICAL, EBUSY, ENOTFOUND, ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7, -8
ADVECTION, BURGERS, EULER = 0, 1, 2
PERIODIC, TRANSMISSIVE = 0, 1
FP64, FP32 = 0, 1
RBF_WENO5, WENO5_JS, RBF_ENO3, ENO3 = 0, 1, 2, 3  # k = 3
RBF_WENO3, WENO3_JS, RBF_ENO2, ENO2 = 4, 5, 6, 7  # k = 2
RBF_ENO2_2D = 8  # k = 2, Section 6 (2D only)
SWITCH_MONOTONE, SWITCH_OFF = 0, 1
COMPONENTWISE, CHARACTERISTIC = 0, 1


class Params(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("dim", ctypes.c_int32), ("flux", ctypes.c_int32),
        ("ncomp", ctypes.c_int32), ("bc", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("recon", ctypes.c_int32), ("switch_mode", ctypes.c_int32),
        ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("speed_x", ctypes.c_double), ("speed_y", ctypes.c_double), ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double), ("eps_weno", ctypes.c_double), ("eps_m", ctypes.c_double),
        ("dt_fixed", ctypes.c_double), ("variables", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double), ("nsteps", ctypes.c_int64), ("alpha", ctypes.c_double * 2),
        ("mass", ctypes.c_double * 4), ("err", ctypes.c_int32), ("err_stage", ctypes.c_int32),
    ]

    def as_dict(self):
        return {"t": self.t, "nsteps": self.nsteps, "alpha": list(self.alpha), "mass": list(self.mass),
                "err": self.err, "err_stage": self.err_stage}


class NpwError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = lib().npweno_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


_lib = None
_VP = ctypes.c_void_p


def lib():
    """Load libnpweno.so (built by __graft_entry__.build() / paper_1602_00182_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        # torch ships its own HIP runtime; load it first so the process has a single one
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(Params)
        S = ctypes.POINTER(Stats)
        L.npweno_abi_version.restype = ctypes.c_int
        L.npweno_strerror.argtypes = [ctypes.c_int]
        L.npweno_strerror.restype = ctypes.c_char_p
        L.npweno_default_params.argtypes = [P]
        L.npweno_create.argtypes = [P, _VP, ctypes.c_int, _VP, ctypes.POINTER(_VP)]
        L.npweno_step.argtypes = [_VP, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
        L.npweno_solve.argtypes = [_VP, ctypes.c_double, ctypes.c_int64, S]
        L.npweno_rhs.argtypes = [_VP, _VP, ctypes.c_int]
        L.npweno_read.argtypes = [_VP, _VP, ctypes.c_int]
        L.npweno_rhs_noalloc.argtypes = [P, _VP, _VP, _VP, _VP]
        L.npweno_write.argtypes = [_VP, _VP, ctypes.c_int, ctypes.c_double]
        L.npweno_get_stats.argtypes = [_VP, S]
        L.npweno_destroy.argtypes = [_VP]
        L.npweno_destroy.restype = None
        L.npweno_create_batch.argtypes = [P, ctypes.c_int32, ctypes.POINTER(_VP), ctypes.c_int, _VP,
                                          ctypes.POINTER(_VP)]
        L.npweno_solve_batch.argtypes = [_VP, ctypes.POINTER(ctypes.c_double), ctypes.c_int64, S]
        L.npweno_read_instance.argtypes = [_VP, ctypes.c_int32, _VP, ctypes.c_int]
        L.npweno_get_stats_instance.argtypes = [_VP, ctypes.c_int32, S]
        L.npweno_instance_count.argtypes = [_VP]
        L.npweno_instance_count.restype = ctypes.c_int
        I32P = ctypes.POINTER(ctypes.c_int32)
        L.npweno_launch_shape.argtypes = [_VP, I32P, I32P, I32P, I32P]
        U64 = ctypes.c_uint64
        L.npw_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, _VP, ctypes.POINTER(_VP)]
        L.npw_server_submit.argtypes = [_VP, P, _VP, ctypes.c_double, ctypes.POINTER(U64)]
        L.npw_server_pump.argtypes = [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32)]
        L.npw_server_poll.argtypes = [_VP, U64, _VP, S]
        L.npw_server_times.argtypes = [_VP, U64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]
        L.npw_server_release.argtypes = [_VP, U64]
        L.npw_server_destroy.argtypes = [_VP]
        L.npw_server_destroy.restype = None
        for name in ("npw_server_create", "npw_server_submit", "npw_server_pump", "npw_server_poll",
                     "npw_server_times", "npw_server_release"):
            getattr(L, name).restype = ctypes.c_int
        for name in ("npweno_create", "npweno_step", "npweno_solve", "npweno_rhs", "npweno_rhs_noalloc", "npweno_read",
                     "npweno_write", "npweno_get_stats", "npweno_create_batch", "npweno_solve_batch",
                     "npweno_read_instance", "npweno_get_stats_instance"):
            getattr(L, name).restype = ctypes.c_int
        if L.npweno_abi_version() != NPW_ABI_VERSION:
            raise RuntimeError("libnpweno.so ABI version mismatch")
        _lib = L
    return _lib


def make_params(**kw) -> Params:
    p = Params()
    lib().npweno_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _check(rc: int, what: str):
    if rc != OK:
        raise NpwError(rc, what)


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _stream_handle(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return ctypes.c_void_p(0)


def _buf(x, dtype):
    """(pointer, on_device, keepalive) for a numpy array or torch CUDA tensor of `dtype`."""
    if _is_torch(x):
        import torch
        tdt = torch.float64 if dtype == np.float64 else torch.float32
        if x.dtype != tdt or not x.is_cuda or not x.is_contiguous():
            raise TypeError(f"expected a contiguous CUDA tensor of {tdt}")
        return ctypes.c_void_p(x.data_ptr()), 1, x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data_as(ctypes.c_void_p), 0, a


def rhs_noalloc(u, L_out, status=None, stream=None, **params):
    """npweno_rhs_noalloc: L(u) of a caller-held device state into L_out (torch CUDA tensors of the
    precision's dtype), enqueued on the stream without allocating; `status` (optional int32 CUDA
    tensor of one element) receives the state check's code.  Returns without synchronizing."""
    p = make_params(**params)
    dtype = np.float64 if p.precision == FP64 else np.float32
    up, udev, _ = _buf(u, dtype)
    lp, ldev, _ = _buf(L_out, dtype)
    if not (udev and ldev):
        raise TypeError("rhs_noalloc takes device tensors")
    n = int(p.ncomp * p.nx * (p.ny if p.dim == 2 else 1))
    if u.numel() != n or L_out.numel() != n:
        raise ValueError(f"u and L_out must hold {n} elements")
    sp = _VP(0)
    if status is not None:
        import torch
        if status.dtype != torch.int32 or not status.is_cuda or status.numel() != 1:
            raise TypeError("status must be a one-element int32 CUDA tensor")
        sp = _VP(status.data_ptr())
    _check(lib().npweno_rhs_noalloc(ctypes.byref(p), up, lp, _stream_handle(stream), sp), "npweno_rhs_noalloc")


class Solver:
    """One grid: create / step / solve / rhs / read / write / stats / destroy."""

    def __init__(self, u0, stream=None, **params):
        self.p = make_params(**params)
        self.dtype = np.float64 if self.p.precision == FP64 else np.float32
        self.size = int(self.p.ncomp * self.p.nx * (self.p.ny if self.p.dim == 2 else 1))
        ptr, dev, keep = _buf(u0, self.dtype)
        if (keep.numel() if dev else keep.size) != self.size:
            raise ValueError(f"u0 has the wrong size (expected {self.size})")
        h = ctypes.c_void_p()
        self._stream = _stream_handle(stream)
        _check(lib().npweno_create(ctypes.byref(self.p), ptr, dev, self._stream, ctypes.byref(h)), "npweno_create")
        self.h = h

    def step(self, t_final: float) -> float:
        dt = ctypes.c_double(0.0)
        _check(lib().npweno_step(self.h, t_final, ctypes.byref(dt)), "npweno_step")
        return dt.value

    def solve(self, t_final: float, max_steps: int = -1) -> dict:
        st = Stats()
        _check(lib().npweno_solve(self.h, t_final, max_steps, ctypes.byref(st)), "npweno_solve")
        return st.as_dict()

    def rhs(self, out=None):
        if out is None:
            out = np.empty(self.size, dtype=self.dtype)
        ptr, dev, keep = _buf(out, self.dtype)
        _check(lib().npweno_rhs(self.h, ptr, dev), "npweno_rhs")
        return keep

    def read(self, out=None):
        if out is None:
            out = np.empty(self.size, dtype=self.dtype)
        ptr, dev, keep = _buf(out, self.dtype)
        _check(lib().npweno_read(self.h, ptr, dev), "npweno_read")
        return keep

    def write(self, u, t: float = 0.0):
        ptr, dev, keep = _buf(u, self.dtype)
        _check(lib().npweno_write(self.h, ptr, dev, t), "npweno_write")

    def stats(self) -> dict:
        st = Stats()
        _check(lib().npweno_get_stats(self.h, ctypes.byref(st)), "npweno_get_stats")
        return st.as_dict()

    def launch_shape(self) -> dict:
        """Stage-kernel launch shape in use: 1D threads per workgroup, 2D owned tile."""
        b, tx, ty, sh = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().npweno_launch_shape(self.h, ctypes.byref(b), ctypes.byref(tx), ctypes.byref(ty),
                                         ctypes.byref(sh)), "npweno_launch_shape")
        return {"block": b.value, "tile_x": tx.value, "tile_y": ty.value, "lds_shared": sh.value}

    def close(self):
        if getattr(self, "h", None):
            lib().npweno_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Several independent 1D instances stepped together (npweno_create_batch)."""

    def __init__(self, states, params_list, stream=None):
        if len(states) != len(params_list) or not states:
            raise ValueError("one parameter set per state")
        n = len(states)
        self.params = (Params * n)()
        for b, kw in enumerate(params_list):
            self.params[b] = make_params(**kw)
        self.dtype = np.float64 if self.params[0].precision == FP64 else np.float32
        self.sizes = [int(p.ncomp * p.nx * (p.ny if p.dim == 2 else 1)) for p in self.params]
        keep, ptrs, dev = [], (_VP * n)(), 0
        for b, u in enumerate(states):
            ptr, d, k = _buf(u, self.dtype)
            if (k.numel() if d else k.size) != self.sizes[b]:
                raise ValueError(f"state {b} has the wrong size")
            ptrs[b] = ptr.value
            dev = d
            keep.append(k)
        h = ctypes.c_void_p()
        self._stream = _stream_handle(stream)
        _check(lib().npweno_create_batch(self.params, n, ptrs, dev, self._stream, ctypes.byref(h)),
               "npweno_create_batch")
        self.h = h
        self.count = n

    def solve(self, t_final, max_steps: int = -1, raise_on_error: bool = True):
        T = (ctypes.c_double * self.count)(*([float(t_final)] * self.count if np.isscalar(t_final) else t_final))
        st = (Stats * self.count)()
        rc = lib().npweno_solve_batch(self.h, T, max_steps, st)
        if rc != OK and raise_on_error:
            raise NpwError(rc, "npweno_solve_batch")
        return [x.as_dict() for x in st], rc

    def read(self, b: int, out=None):
        if out is None:
            out = np.empty(self.sizes[b], dtype=self.dtype)
        ptr, dev, keep = _buf(out, self.dtype)
        _check(lib().npweno_read_instance(self.h, b, ptr, dev), "npweno_read_instance")
        return keep

    def stats(self, b: int) -> dict:
        st = Stats()
        _check(lib().npweno_get_stats_instance(self.h, b, ctypes.byref(st)), "npweno_get_stats_instance")
        return st.as_dict()

    launch_shape = Solver.launch_shape

    def close(self):
        if getattr(self, "h", None):
            lib().npweno_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """Continuous-batching request loop (npw_server_*): submit, pump, poll."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 256, precision: int = FP32, stream=None):
        h = ctypes.c_void_p()
        self.precision = precision
        self.dtype = np.float64 if precision == FP64 else np.float32
        _check(lib().npw_server_create(int(hbm_budget_bytes), max_slots, precision, _stream_handle(stream),
                                       ctypes.byref(h)), "npw_server_create")
        self.h = h
        self.sizes = {}

    def submit(self, u0, t_final: float, **params) -> int:
        params.setdefault("precision", self.precision)
        p = make_params(**params)
        a = np.ascontiguousarray(u0, dtype=self.dtype)
        rid = ctypes.c_uint64()
        _check(lib().npw_server_submit(self.h, ctypes.byref(p), a.ctypes.data_as(_VP), float(t_final),
                                       ctypes.byref(rid)), "npw_server_submit")
        self.sizes[rid.value] = a.size
        return rid.value

    def pump(self, steps: int = 16):
        nr, nq = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().npw_server_pump(self.h, steps, ctypes.byref(nr), ctypes.byref(nq)), "npw_server_pump")
        return nr.value, nq.value

    def poll(self, rid: int):
        """None while running; (state, stats, rc) once finished (rc is the request's error code)."""
        out = np.empty(self.sizes[rid], dtype=self.dtype)
        st = Stats()
        rc = lib().npw_server_poll(self.h, rid, out.ctypes.data_as(_VP), ctypes.byref(st))
        if rc == EBUSY:
            return None
        if rc == ENOTFOUND or rc == EINVAL:
            raise NpwError(rc, "npw_server_poll")
        return out, st.as_dict(), rc

    def times(self, rid: int):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        lib().npw_server_times(self.h, rid, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return a.value, b.value, c.value

    def finished(self, rid: int) -> bool:
        """True once the request has finished (npw_server_times stops returning NPW_EBUSY); copies
        nothing."""
        rc = lib().npw_server_times(self.h, rid, None, None, None)
        if rc not in (OK, EBUSY):
            raise NpwError(rc, "npw_server_times")
        return rc == OK

    def release(self, rid: int):
        lib().npw_server_release(self.h, rid)

    def close(self):
        if getattr(self, "h", None):
            lib().npw_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def workload_params(w, precision=FP64) -> dict:
    """Solver keyword arguments for an inputs.Workload."""
    d = w.params()
    d["precision"] = precision
    if d["dim"] == 1:
        d["ny"] = 1
    return d
