"""Seeded synthetic inputs shaped like the paper's workloads.

This module only builds initial cell averages and problem descriptions; it holds none of the
scheme's arithmetic.  The same arrays feed the HIP library and the CPU oracle.

Workloads (all on uniform grids, cell averages in component-major layout u[c*ncell + k]):

* ``advection_sine``   -- u_t + u_x = 0 on [-1, 1], periodic, u0 = sin(pi x) (Section 5.2,
  Example 1 of the paper; the N = 80, CFL 0.5, T = 2 case is the small parity workload).
* ``burgers_noisy``    -- u_t + (u^2/2)_x = 0 on [-1, 1], periodic, u0 = 0.5 + sin(pi x) plus
  seeded i.i.d. U(-1e-3, 1e-3) per cell, run past shock formation to T = 1.5/pi
  (N = 65536 is the headline throughput workload).
* ``euler_riemann_batch`` -- 1D Euler (gamma 1.4) Riemann problems on [-1, 1], jump at x = 0,
  transmissive, left/right (rho, u, p) in U[0.1,1] x U[-1,1] x U[0.1,1], N in U{256..4096}.
* ``serving_trace``    -- Poisson arrivals of mixed advection/Burgers/Euler requests with
  log-uniform N in [256, 262144] and smooth-plus-step data.
* ``euler2d_quadrants`` -- 2D Euler on [0,1]^2 split at (0.5, 0.5) into four seeded constant
  states, transmissive.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

ADVECTION, BURGERS, EULER = 0, 1, 2
PERIODIC, TRANSMISSIVE = 0, 1
RBF_WENO5, WENO5_JS, RBF_ENO3, ENO3 = 0, 1, 2, 3  # k = 3 (Table 3)
RBF_WENO3, WENO3_JS, RBF_ENO2, ENO2 = 4, 5, 6, 7  # k = 2 (Table 2)
RBF_ENO2_2D = 8  # k = 2, Section 6 (2D only)
SWITCH_MONOTONE, SWITCH_OFF = 0, 1
COMPONENTWISE, CHARACTERISTIC = 0, 1


@dataclass
class Workload:
    """One solve: problem parameters plus initial cell averages (float64)."""
    name: str
    nx: int
    flux: int
    u0: np.ndarray
    T: float
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
    variables: int = COMPONENTWISE
    meta: dict = field(default_factory=dict)

    @property
    def ncell(self) -> int:
        return self.nx * (self.ny if self.dim == 2 else 1)

    @property
    def dx(self) -> float:
        return (self.x1 - self.x0) / self.nx

    def params(self) -> dict:
        """Problem parameters as plain keyword values (no initial data)."""
        keys = ("dim", "flux", "ncomp", "nx", "ny", "x0", "x1", "y0", "y1", "bc", "speed_x", "speed_y",
                "gamma", "cfl", "eps_weno", "eps_m", "recon", "switch_mode", "dt_fixed", "variables")
        return {k: getattr(self, k) for k in keys}

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def cell_centers(n: int, x0: float, x1: float) -> np.ndarray:
    h = (x1 - x0) / n
    return x0 + (np.arange(n) + 0.5) * h


def sine_cell_averages(n: int, x0: float = -1.0, x1: float = 1.0, k: float = math.pi,
                       phase: float = 0.0) -> np.ndarray:
    """Exact cell averages of sin(k x + phase), in the cancellation-free form
    sin(k x_i + phase) * sin(k h / 2) / (k h / 2)."""
    h = (x1 - x0) / n
    xc = cell_centers(n, x0, x1)
    s = k * h / 2.0
    return np.sin(k * xc + phase) * (math.sin(s) / s)


def advection_sine(n: int = 80, T: float = 2.0, cfl: float = 0.5, **kw) -> Workload:
    u0 = sine_cell_averages(n)
    return Workload(name=f"advection_sine_N{n}", nx=n, flux=ADVECTION, u0=u0, T=T, cfl=cfl, **kw)


def burgers_noisy(n: int = 65536, seed: int = 2, T: float = 1.5 / math.pi, cfl: float = 0.5,
                  noise: float = 1e-3, **kw) -> Workload:
    rng = np.random.Generator(np.random.PCG64(seed))
    u0 = 0.5 + sine_cell_averages(n) + rng.uniform(-noise, noise, size=n)
    return Workload(name=f"burgers_noisy_N{n}", nx=n, flux=BURGERS, u0=u0, T=T, cfl=cfl, **kw)


def burgers_sine(n: int, T: float = 0.2, cfl: float = 0.5, **kw) -> Workload:
    """Section 5.2, Example 3: u0 = -sin(pi x) on [-1, 1], periodic."""
    u0 = -sine_cell_averages(n)
    return Workload(name=f"burgers_sine_N{n}", nx=n, flux=BURGERS, u0=u0, T=T, cfl=cfl, **kw)


def euler_prim_to_cons(rho, u, p, gamma=1.4, v=None):
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    if v is None:
        return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])
    v = np.asarray(v, dtype=np.float64)
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def riemann_cell_averages(n: int, left, right, gamma: float = 1.4, x0: float = -1.0,
                          x1: float = 1.0, xs: float = 0.0) -> np.ndarray:
    """Cell averages (3 x n, conservative) of a 1D Riemann state with the jump at xs; the cell
    that straddles the jump gets the exact length-weighted average of the two states."""
    UL = euler_prim_to_cons(*left, gamma=gamma)
    UR = euler_prim_to_cons(*right, gamma=gamma)
    h = (x1 - x0) / n
    xl = x0 + np.arange(n) * h
    frac_left = np.clip((xs - xl) / h, 0.0, 1.0)
    return UL[:, None] * frac_left[None, :] + UR[:, None] * (1.0 - frac_left[None, :])


def sod(n: int = 600, T: float = 0.2, cfl: float = 0.5, **kw) -> Workload:
    """Section 5.2, Example 4: Sod's shock tube on [-1, 1] (jump at 0), transmissive."""
    u0 = riemann_cell_averages(n, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)).reshape(-1)
    return Workload(name=f"sod_N{n}", nx=n, flux=EULER, ncomp=3, u0=u0, T=T, cfl=cfl, bc=TRANSMISSIVE, **kw)


def euler_riemann_batch(count: int = 4096, seed: int = 3, nmin: int = 256, nmax: int = 4096,
                        T: float = 0.2, cfl: float = 0.5, gamma: float = 1.4):
    """Batch of 1D Euler Riemann problems (one Workload per instance)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        L = (rng.uniform(0.1, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 1.0))
        R = (rng.uniform(0.1, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 1.0))
        u0 = riemann_cell_averages(n, L, R, gamma=gamma).reshape(-1)
        out.append(Workload(name=f"riemann_{b}", nx=n, flux=EULER, ncomp=3, u0=u0, T=T, cfl=cfl,
                            bc=TRANSMISSIVE, gamma=gamma, meta={"left": L, "right": R}))
    return out


def euler2d_quadrants(n: int = 2048, seed: int = 5, T: float = 0.25, cfl: float = 0.4,
                      gamma: float = 1.4) -> Workload:
    """2D Euler on [0,1]^2, four seeded constant states split at (0.5, 0.5), transmissive.
    Quadrant q = 2*(y > 0.5) + (x > 0.5)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    states = []
    for _ in range(4):
        rho = rng.uniform(0.1, 1.5)
        p = rng.uniform(0.1, 1.5)
        u = rng.uniform(-1.0, 1.0)
        v = rng.uniform(-1.0, 1.0)
        states.append((rho, u, v, p))
    xc = cell_centers(n, 0.0, 1.0)
    q = (xc[None, :] > 0.5).astype(int) + 2 * (xc[:, None] > 0.5).astype(int)  # [j, i]
    prim = np.array(states)  # 4 x (rho, u, v, p)
    rho = prim[q, 0]
    u = prim[q, 1]
    v = prim[q, 2]
    p = prim[q, 3]
    U = euler_prim_to_cons(rho, u, p, gamma=gamma, v=v)  # 4 x ny x nx
    return Workload(name=f"euler2d_quadrants_{n}", nx=n, ny=n, dim=2, flux=EULER, ncomp=4,
                    u0=U.reshape(-1), T=T, cfl=cfl, bc=TRANSMISSIVE, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                    gamma=gamma, meta={"states": states})


def advection2d_sine(n: int = 2048, T: float = 0.25, cfl: float = 0.4, **kw) -> Workload:
    """Section 6's test problem: v_t + v_x + v_y = 0 on [0,1]^2, periodic, v0 = sin(2 pi (x + y)).
    Exact cell averages: sin(2 pi (x_i + y_j)) * s^2 with s = sin(pi h) / (pi h), because the
    average of exp(2 pi i x) over a cell is exp(2 pi i x_i) s."""
    h = 1.0 / n
    xc = cell_centers(n, 0.0, 1.0)
    s = math.sin(math.pi * h) / (math.pi * h)
    u0 = np.sin(2.0 * math.pi * (xc[None, :] + xc[:, None])) * (s * s)  # [j, i]
    return Workload(name=f"advection2d_sine_{n}", nx=n, ny=n, dim=2, flux=ADVECTION, u0=u0.reshape(-1), T=T,
                    cfl=cfl, x0=0.0, x1=1.0, y0=0.0, y1=1.0, speed_x=1.0, speed_y=1.0, **kw)


def smooth_plus_step(n: int, kind: int, rng: np.random.Generator, gamma: float = 1.4) -> np.ndarray:
    """Serving-trace initial data: A sin(pi k x + phi) + B H(x - xs) on [-1, 1] for scalars; Euler
    gets rho = 1 + 0.3 (same shape), p = 1 + 0.3 (same shape), u = 0.2 sin(pi x)."""
    A = rng.uniform(0.2, 1.0)
    k = int(rng.integers(1, 4))
    B = rng.uniform(-0.5, 0.5)
    xs = rng.uniform(-0.5, 0.5)
    phi = rng.uniform(0.0, 2 * math.pi)
    h = 2.0 / n
    xl = -1.0 + np.arange(n) * h
    frac_right = np.clip((xl + h - xs) / h, 0.0, 1.0)  # part of the cell beyond the step
    shape = A * sine_cell_averages(n, k=math.pi * k, phase=phi) + B * frac_right
    if kind != EULER:
        return shape
    rho = 1.0 + 0.3 * shape
    p = 1.0 + 0.3 * shape
    u = 0.2 * sine_cell_averages(n)
    # cell averages of the conservative variables, formed from the primitive cell values
    return euler_prim_to_cons(rho, u, p, gamma=gamma).reshape(-1)


@dataclass
class Request:
    rid: int
    arrival: float
    work: Workload


def serving_trace(nreq: int = 2000, rate: float = 2000.0, seed: int = 4, nmin: int = 256,
                  nmax: int = 262144, cfl: float = 0.5):
    """Poisson arrivals at `rate` req/s; kind uniform over {advection, Burgers, Euler};
    N = floor(exp(U(ln nmin, ln nmax))); T ~ U[0.1, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for r in range(nreq):
        t += rng.exponential(1.0 / rate)
        kind = int(rng.integers(0, 3))
        n = int(math.floor(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        T = float(rng.uniform(0.1, 1.0))
        u0 = smooth_plus_step(n, kind, rng)
        if kind == EULER:
            w = Workload(name=f"req{r}", nx=n, flux=EULER, ncomp=3, u0=u0, T=T, cfl=cfl, bc=TRANSMISSIVE)
        else:
            w = Workload(name=f"req{r}", nx=n, flux=kind, u0=u0, T=T, cfl=cfl, bc=PERIODIC)
        out.append(Request(r, t, w))
    return out
