"""FP64 CPU oracle of the non-polynomial (MQ-RBF perturbed) ENO/WENO finite-volume schemes:
k = 3 (Table 3) and k = 2 (Table 2) in 1D and dimension by dimension in 2D, the two-dimensional
k = 2 reconstruction of Section 6, and characteristic-wise Euler reconstruction.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the product library never does.  The arithmetic lives
in ``npw_oracle.c`` (plain C, IEEE double, no FP contraction); this module compiles it with
gcc and marshals numpy arrays through ctypes.

Every numerical function is pinned by ``tests/test_oracle_*.py`` against something other than
itself (brute-force RBF interpolation, closed forms, the paper's printed error tables, exact
solutions).  See the header of ``npw_oracle.c`` for the passages each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "npw_oracle.c")
_LIB = os.path.join(_HERE, "libnpw_oracle.so")

ADVECTION, BURGERS, EULER = 0, 1, 2
PERIODIC, TRANSMISSIVE = 0, 1
RBF_WENO5, WENO5_JS, RBF_ENO3, ENO3 = 0, 1, 2, 3
RBF_WENO3, WENO3_JS, RBF_ENO2, ENO2 = 4, 5, 6, 7
RBF_ENO2_2D = 8  # Section 6 reconstruction (2D only)
SWITCH_MONOTONE, SWITCH_OFF = 0, 1
OK, EINVAL, ENONFINITE, ENONPHYSICAL = 0, -1, -4, -5


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("flux", ctypes.c_int), ("ncomp", ctypes.c_int), ("bc", ctypes.c_int),
        ("nx", ctypes.c_long), ("ny", ctypes.c_long),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("speed_x", ctypes.c_double), ("speed_y", ctypes.c_double), ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double), ("eps_weno", ctypes.c_double), ("eps_m", ctypes.c_double),
        ("recon", ctypes.c_int), ("switch_mode", ctypes.c_int), ("dt_fixed", ctypes.c_double),
        ("charwise", ctypes.c_int),
    ]


@dataclass
class Problem:
    """Problem description for the oracle (the oracle's own mirror of the solver parameters)."""
    nx: int
    flux: int = ADVECTION
    dim: int = 1
    ny: int = 1
    ncomp: int = 1
    bc: int = PERIODIC
    x0: float = -1.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    speed_x: float = 1.0
    speed_y: float = 0.0
    gamma: float = 1.4
    cfl: float = 0.5
    eps_weno: float = 1e-6
    eps_m: float = 1e-12
    recon: int = RBF_WENO5
    switch_mode: int = SWITCH_MONOTONE
    dt_fixed: float = 0.0
    charwise: int = 0

    def c(self) -> _Problem:
        return _Problem(self.dim, self.flux, self.ncomp, self.bc, self.nx, self.ny if self.dim == 2 else 1,
                        self.x0, self.x1, self.y0, self.y1, self.speed_x, self.speed_y, self.gamma,
                        self.cfl, self.eps_weno, self.eps_m, self.recon, self.switch_mode, self.dt_fixed,
                        self.charwise)

    @property
    def ncell(self) -> int:
        return self.nx * (self.ny if self.dim == 2 else 1)

    @property
    def dx(self) -> float:
        return (self.x1 - self.x0) / self.nx


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Problem)
        L.npo_table3.argtypes = [_D, _D]
        L.npo_row_value.argtypes = [ctypes.c_int] + [ctypes.c_double] * 4
        L.npo_row_value.restype = ctypes.c_double
        L.npo_eta.argtypes = [ctypes.c_double] * 5
        L.npo_eta.restype = ctypes.c_double
        L.npo_monotone_flag.argtypes = [ctypes.c_double] * 3
        L.npo_monotone_flag.restype = ctypes.c_int
        L.npo_beta.argtypes = [_D, _D]
        L.npo_recon_minus.argtypes = [_D, ctypes.c_double, ctypes.c_double]
        L.npo_recon_minus.restype = ctypes.c_double
        L.npo_recon_plus.argtypes = [_D, ctypes.c_double, ctypes.c_double]
        L.npo_recon_plus.restype = ctypes.c_double
        L.npo_eno_stencil.argtypes = [_D]
        L.npo_eno_stencil.restype = ctypes.c_int
        L.npo_eno_minus.argtypes = [_D, ctypes.c_double]
        L.npo_eno_minus.restype = ctypes.c_double
        L.npo_eno_plus.argtypes = [_D, ctypes.c_double]
        L.npo_eno_plus.restype = ctypes.c_double
        L.npo_row2_value.argtypes = [ctypes.c_int] + [ctypes.c_double] * 3
        L.npo_row2_value.restype = ctypes.c_double
        L.npo_eta2.argtypes = [ctypes.c_double] * 4
        L.npo_eta2.restype = ctypes.c_double
        L.npo_line_states.argtypes = [P, _D, ctypes.c_long, _D, _D, _D, _I]
        L.npo_char_basis.argtypes = [P, ctypes.c_int, _D, _D, _D, _D, _D]
        L.npo_char_interface.argtypes = [P, ctypes.c_int, _D, _D, _D]
        L.npo_cross_edge.argtypes = [_D, _D, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.npo_cross_edge.restype = ctypes.c_double
        L.npo_face_states.argtypes = [P, ctypes.c_int, _D, _D, _D]
        L.npo_alpha.argtypes = [P, _D, _D]
        L.npo_alpha.restype = ctypes.c_int
        L.npo_rhs.argtypes = [P, _D, _D, _D]
        L.npo_rhs.restype = ctypes.c_int
        L.npo_step.argtypes = [P, _D, ctypes.c_double, _D, _D]
        L.npo_step.restype = ctypes.c_int
        L.npo_solve.argtypes = [P, _D, ctypes.c_double, ctypes.c_long, _D, ctypes.POINTER(ctypes.c_long)]
        L.npo_solve.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def table3():
    c = np.zeros(12)
    p = np.zeros(12)
    lib().npo_table3(_dp(c), _dp(p))
    return c.reshape(4, 3), p.reshape(4, 3)


def row_value(r: int, w0: float, w1: float, w2: float, eta: float) -> float:
    return lib().npo_row_value(r, w0, w1, w2, eta)


def eta(um1, u0, up1, up2, eps_m=1e-12) -> float:
    return lib().npo_eta(um1, u0, up1, up2, eps_m)


def monotone_flag(um1, u0, up1) -> int:
    return lib().npo_monotone_flag(um1, u0, up1)


def beta(u5) -> np.ndarray:
    u5 = _f64(u5)
    b = np.zeros(3)
    lib().npo_beta(_dp(u5), _dp(b))
    return b


def recon_minus(u5, eta_right, eps=1e-6) -> float:
    u5 = _f64(u5)
    return lib().npo_recon_minus(_dp(u5), eta_right, eps)


def recon_plus(u5, eta_left, eps=1e-6) -> float:
    u5 = _f64(u5)
    return lib().npo_recon_plus(_dp(u5), eta_left, eps)


def eno_stencil(u5) -> int:
    u5 = _f64(u5)
    return lib().npo_eno_stencil(_dp(u5))


def eno_minus(u5, eta_right) -> float:
    return lib().npo_eno_minus(_dp(_f64(u5)), eta_right)


def eno_plus(u5, eta_left) -> float:
    return lib().npo_eno_plus(_dp(_f64(u5)), eta_left)


def row2_value(r: int, w0: float, w1: float, eta: float) -> float:
    return lib().npo_row2_value(r, w0, w1, eta)


def eta2(um1, u0, up1, eps_m=1e-12) -> float:
    return lib().npo_eta2(um1, u0, up1, eps_m)


def line_states(pb: Problem, line):
    """(v^-, v^+, eta, flag) at the n+1 interfaces x_{i+1/2}, i = -1..n-1, of one grid line."""
    line = _f64(line)
    n = line.size
    vm, vp, et = np.zeros(n + 1), np.zeros(n + 1), np.zeros(n + 1)
    fl = np.zeros(n + 1, dtype=np.int32)
    cp = pb.c()
    lib().npo_line_states(ctypes.byref(cp), _dp(line), n, _dp(vm), _dp(vp), _dp(et),
                          fl.ctypes.data_as(_I))
    return vm, vp, et, fl


class OracleError(RuntimeError):
    def __init__(self, rc):
        super().__init__(f"oracle returned {rc}")
        self.rc = rc


def char_basis(pb: Problem, direction: int, UL, UR):
    """(Lm, Rm, lam) of the Euler flux Jacobian along `direction` at the Roe average of UL, UR:
    rows of Lm are left eigenvectors, columns of Rm right eigenvectors."""
    m = pb.ncomp
    UL, UR = _f64(UL).copy(), _f64(UR).copy()
    Lm, Rm, lam = np.zeros(m * m), np.zeros(m * m), np.zeros(m)
    p = pb.c()
    rc = lib().npo_char_basis(ctypes.byref(p), direction, _dp(UL), _dp(UR), _dp(Lm), _dp(Rm), _dp(lam))
    if rc:
        raise OracleError(rc)
    return Lm.reshape(m, m), Rm.reshape(m, m), lam


def char_interface(pb: Problem, direction: int, U6):
    """(v^-, v^+) at one interface from its six-cell window U6[k, c] (cells i-2..i+3),
    characteristic-wise."""
    m = pb.ncomp
    U6 = _f64(U6).reshape(6, m).copy()
    vm, vp = np.zeros(m), np.zeros(m)
    p = pb.c()
    rc = lib().npo_char_interface(ctypes.byref(p), direction, _dp(U6), _dp(vm), _dp(vp))
    if rc:
        raise OracleError(rc)
    return vm, vp


def cross_edge(w3, t2, right_edge: bool, use_switch: bool = True, eps_m: float = 1e-12) -> float:
    """Section 6 edge value of a cell from its along-sweep window w3 and transverse neighbours t2."""
    w3, t2 = _f64(w3).copy(), _f64(t2).copy()
    return lib().npo_cross_edge(_dp(w3), _dp(t2), int(right_edge), int(use_switch), eps_m)


def face_states(pb: Problem, direction: int, field):
    """Section 6 edge states (v^-, v^+) of one component field (ny x nx) along `direction`:
    arrays of shape (lines, n + 1), interface f between cells f-1 and f."""
    field = _f64(field).reshape(-1).copy()
    n, lines = (pb.nx, pb.ny) if direction == 0 else (pb.ny, pb.nx)
    vm, vp = np.zeros(lines * (n + 1)), np.zeros(lines * (n + 1))
    p = pb.c()
    rc = lib().npo_face_states(ctypes.byref(p), direction, _dp(field), _dp(vm), _dp(vp))
    if rc:
        raise OracleError(rc)
    return vm.reshape(lines, n + 1), vp.reshape(lines, n + 1)


def alpha(pb: Problem, u):
    u = _f64(u)
    a = np.zeros(2)
    cp = pb.c()
    rc = lib().npo_alpha(ctypes.byref(cp), _dp(u), _dp(a))
    if rc:
        raise OracleError(rc)
    return a


def rhs(pb: Problem, u):
    u = _f64(u).copy()
    L = np.zeros_like(u)
    a = np.zeros(2)
    cp = pb.c()
    rc = lib().npo_rhs(ctypes.byref(cp), _dp(u), _dp(L), _dp(a))
    if rc:
        raise OracleError(rc)
    return L, a


def step(pb: Problem, u, T: float, t: float = 0.0):
    """One SSP-RK3 step; returns (u_new, t_new, dt)."""
    u = _f64(u).copy()
    tt = ctypes.c_double(t)
    dt = ctypes.c_double(0.0)
    cp = pb.c()
    rc = lib().npo_step(ctypes.byref(cp), _dp(u), T, ctypes.byref(tt), ctypes.byref(dt))
    if rc:
        raise OracleError(rc)
    return u, tt.value, dt.value


def solve(pb: Problem, u, T: float, t: float = 0.0, max_steps: int = -1):
    """Run SSP-RK3 steps until T; returns (u, t, nsteps)."""
    u = _f64(u).copy()
    tt = ctypes.c_double(t)
    ns = ctypes.c_long(0)
    cp = pb.c()
    rc = lib().npo_solve(ctypes.byref(cp), _dp(u), T, max_steps, ctypes.byref(tt), ctypes.byref(ns))
    if rc:
        raise OracleError(rc)
    return u, tt.value, ns.value


def errors(u, exact):
    """L1 = mean|e|, L2 = sqrt(mean e^2), Linf = max|e| over cell averages."""
    e = np.abs(np.asarray(u, dtype=np.float64) - np.asarray(exact, dtype=np.float64))
    return float(e.mean()), float(np.sqrt((e * e).mean())), float(e.max())
