"""The allocation-free right-hand side (npweno_rhs_noalloc) against npweno_rhs of a solver on the
same state: bit for bit, two calls in a row with the second on a smaller grid (the fixed scratch
keeps the previous call's contents), both precisions, 1D and 2D, and the status of a bad state."""
import sys

import numpy as np
import pytest

from paper_1602_00182_amd import binding as B
from paper_1602_00182_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _burgers(n):
    return I.burgers_noisy(n=n, seed=n % 97)


def _euler2d(nx, ny):
    w = I.euler2d_quadrants(n=max(nx, ny), seed=5)
    U = w.u0.reshape(4, w.ny, w.nx)[:, :ny, :nx].copy().reshape(-1)
    return w.with_(nx=nx, ny=ny, u0=U)


def _one(w, prec):
    import torch
    tdt = torch.float32 if prec == B.FP32 else torch.float64
    prm = B.workload_params(w, prec)
    u = torch.tensor(w.u0, dtype=tdt, device="cuda")
    L = torch.full_like(u, float("nan"))
    status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    B.rhs_noalloc(u, L, status, **prm)
    torch.cuda.synchronize()
    got = L.cpu().numpy()
    with B.Solver(u, **prm) as s:
        want = s.rhs()
    assert int(status.item()) == B.OK
    assert np.array_equal(got, want), float(np.nanmax(np.abs(got - want)))


# each pair: a larger grid, then a smaller one (same or other kind), through the shared scratch
PAIRS = [
    ("burgers 1D fp64 200000 -> 777", lambda: _burgers(200000), lambda: _burgers(777), B.FP64),
    ("burgers 1D fp32 300001 -> 64", lambda: _burgers(300001), lambda: _burgers(64), B.FP32),
    ("euler 1D char fp32 -> burgers", lambda: I.sod(5000).with_(variables=I.CHARACTERISTIC),
     lambda: _burgers(1000), B.FP32),
    ("euler 2D fp32 700x300 -> 70x13", lambda: _euler2d(700, 300), lambda: _euler2d(70, 13), B.FP32),
    ("euler 2D fp64 257x129 -> 9x5", lambda: _euler2d(257, 129), lambda: _euler2d(9, 5), B.FP64),
    ("advection 2D section 6 fp32 -> 1D rbf_weno3", lambda: I.advection2d_sine(n=200).with_(recon=I.RBF_ENO2_2D),
     lambda: I.advection_sine(n=300).with_(recon=I.RBF_WENO3), B.FP32),
]


@pytest.mark.parametrize("name,first,second,prec", PAIRS, ids=[p[0] for p in PAIRS])
def test_noalloc_rhs_equals_solver_rhs_twice(name, first, second, prec, monkeypatch):
    monkeypatch.setenv("NPW_BLOCK", "128")
    monkeypatch.setenv("NPW_TILE2D", "4")
    _say(f"noalloc {name}")
    _one(first(), prec)
    _one(second(), prec)


@pytest.mark.parametrize("scheme", [I.SWITCH_MONOTONE, I.SWITCH_OFF])
def test_noalloc_on_the_strip_shape_equals_solver_fp32(scheme, monkeypatch):
    """With the 62 x 16 column strip asked for, both entry points run the same strip kernel: the
    one built for RBF-WENO5 with the switch, or the one that reads the scheme from the record."""
    monkeypatch.setenv("NPW_BLOCK", "128")
    monkeypatch.setenv("NPW_TILE2D", "6")
    _say(f"noalloc strip switch={scheme}")
    _one(_euler2d(300, 170).with_(switch_mode=scheme), B.FP32)
    _one(_euler2d(70, 13).with_(switch_mode=scheme), B.FP32)


def test_noalloc_reports_a_bad_state_and_leaves_the_output():
    import torch
    _say("noalloc status of a non-finite state")
    w = _burgers(3000)
    u0 = w.u0.copy()
    u0[1234] = np.nan
    u = torch.tensor(u0, dtype=torch.float64, device="cuda")
    L = torch.full_like(u, 7.0)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    B.rhs_noalloc(u, L, status, **B.workload_params(w, B.FP64))
    torch.cuda.synchronize()
    assert int(status.item()) == B.ENONFINITE
    assert bool(torch.all(L == 7.0))
    _one(_burgers(2000), B.FP64)  # the next call starts from a clean record
