"""GPU parity of the Section 6 reconstruction (k = 2, shape parameter from the five-cell cross of
each cell) in the 2D stage kernel against the FP64 oracle."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_1602_00182_amd import binding as B
from paper_1602_00182_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _problem(w):
    return O.Problem(nx=w.nx, flux=w.flux, dim=w.dim, ny=w.ny, ncomp=w.ncomp, bc=w.bc, x0=w.x0, x1=w.x1, y0=w.y0,
                     y1=w.y1, speed_x=w.speed_x, speed_y=w.speed_y, gamma=w.gamma, cfl=w.cfl, eps_weno=w.eps_weno,
                     eps_m=w.eps_m, recon=w.recon, switch_mode=w.switch_mode, dt_fixed=w.dt_fixed)


def _sine(nx, ny, flux=I.ADVECTION, offset=0.0, **kw):
    xc = (np.arange(nx) + 0.5) / nx
    yc = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(xc, yc)
    u0 = offset + np.sin(2 * math.pi * (X + Y))
    return I.Workload(name="s6", nx=nx, ny=ny, dim=2, flux=flux, u0=u0.reshape(-1), T=0.5, x0=0.0, x1=1.0,
                      y0=0.0, y1=1.0, speed_x=1.0, speed_y=1.0, recon=I.RBF_ENO2_2D, **kw)


@pytest.mark.parametrize("flux,offset", [(I.ADVECTION, 0.0), (I.BURGERS, 1.5)])
@pytest.mark.parametrize("sw", [I.SWITCH_MONOTONE, I.SWITCH_OFF])
@pytest.mark.parametrize("shape", [1, 4])
def test_scalar_rhs_and_steps_fp64(flux, offset, sw, shape, monkeypatch):
    _say(f"section6 scalar flux={flux} sw={sw} shape={shape}")
    monkeypatch.setenv("NPW_TILE2D", str(shape))
    w = _sine(97, 41, flux, offset, switch_mode=sw, bc=I.PERIODIC)
    with B.Solver(w.u0, **B.workload_params(w, B.FP64)) as s:
        L = s.rhs()
        s.solve(w.T, max_steps=6)
        u = s.read()
    Lo, _ = O.rhs(_problem(w), w.u0)
    assert np.array_equal(L, Lo)
    uo, _, _ = O.solve(_problem(w), w.u0, w.T, max_steps=6)
    assert np.array_equal(u, uo)


def test_euler_quadrants_fp64():
    _say("section6 euler quadrants")
    base = I.euler2d_quadrants(n=70, seed=5)
    w = base.with_(ny=53, u0=base.u0.reshape(4, 70, 70)[:, :53, :].reshape(-1), recon=I.RBF_ENO2_2D)
    with B.Solver(w.u0, **B.workload_params(w, B.FP64)) as s:
        L = s.rhs()
        s.solve(w.T, max_steps=5)
        u = s.read()
    Lo, _ = O.rhs(_problem(w), w.u0)
    assert np.array_equal(L, Lo)
    uo, _, _ = O.solve(_problem(w), w.u0, w.T, max_steps=5)
    assert np.array_equal(u, uo)


def test_advection_example1_fp32():
    """Section 7, Example 1 setup (dt = 0.1 h, T = 0.5, switch on) at N = 64 in float bulk."""
    _say("section6 advection fp32")
    n = 64
    w = _sine(n, n, switch_mode=I.SWITCH_MONOTONE, bc=I.PERIODIC, dt_fixed=0.1 / n)
    u32 = np.asarray(w.u0, np.float32)
    with B.Solver(u32, **B.workload_params(w, B.FP32)) as s:
        s.solve(w.T)
        u = s.read().astype(np.float64)
    uo, _, _ = O.solve(_problem(w), u32.astype(np.float64), w.T)
    assert np.mean(np.abs(u - uo)) <= 1e-5
    assert np.max(np.abs(u - uo)) <= 1e-4


def test_rejected_in_1d_and_with_characteristic_variables():
    w1 = I.advection_sine(64, recon=I.RBF_ENO2_2D)
    with pytest.raises(B.NpwError) as ei:
        B.Solver(w1.u0, **B.workload_params(w1, B.FP64))
    assert ei.value.code == B.EINVAL
    base = I.euler2d_quadrants(n=16, seed=5)
    w2 = base.with_(recon=I.RBF_ENO2_2D, variables=I.CHARACTERISTIC)
    with pytest.raises(B.NpwError) as ei:
        B.Solver(w2.u0, **B.workload_params(w2, B.FP64))
    assert ei.value.code == B.EINVAL
