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

NPW_ABI_VERSION = 1
OK, EINVAL, ENOMEM, EHIP, ENONFINITE, ENONPHYSICAL, EBUSY, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6, -7
ADVECTION, BURGERS, EULER = 0, 1, 2
PERIODIC, TRANSMISSIVE = 0, 1
FP64, FP32 = 0, 1
RBF_WENO5, WENO5_JS = 0, 1
SWITCH_MONOTONE, SWITCH_OFF = 0, 1


class Params(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("dim", ctypes.c_int32), ("flux", ctypes.c_int32),
        ("ncomp", ctypes.c_int32), ("bc", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("recon", ctypes.c_int32), ("switch_mode", ctypes.c_int32),
        ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("speed_x", ctypes.c_double), ("speed_y", ctypes.c_double), ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double), ("eps_weno", ctypes.c_double), ("eps_m", ctypes.c_double),
        ("dt_fixed", ctypes.c_double),
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
        L.npweno_write.argtypes = [_VP, _VP, ctypes.c_int, ctypes.c_double]
        L.npweno_get_stats.argtypes = [_VP, S]
        L.npweno_destroy.argtypes = [_VP]
        L.npweno_destroy.restype = None
        for name in ("npweno_create", "npweno_step", "npweno_solve", "npweno_rhs", "npweno_read",
                     "npweno_write", "npweno_get_stats"):
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


def workload_params(w, precision=FP64) -> dict:
    """Solver keyword arguments for an inputs.Workload."""
    d = w.params()
    d["precision"] = precision
    if d["dim"] == 1:
        d["ny"] = 1
    return d
