"""GPU batches (one stage launch for many ragged instances): every instance must give exactly
what it gives when solved alone, and agree with the FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle as O
from conftest import assert_fp32_close, check_sums, smooth_cells
from paper_1602_00182_amd import binding as B
from paper_1602_00182_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _oracle_problem(w):
    return O.Problem(nx=w.nx, flux=w.flux, dim=w.dim, ny=w.ny, ncomp=w.ncomp, bc=w.bc, x0=w.x0, x1=w.x1,
                     y0=w.y0, y1=w.y1, speed_x=w.speed_x, speed_y=w.speed_y, gamma=w.gamma, cfl=w.cfl,
                     eps_weno=w.eps_weno, eps_m=w.eps_m, recon=w.recon, switch_mode=w.switch_mode,
                     dt_fixed=w.dt_fixed)


def _states(ws, prec):
    dt = np.float64 if prec == B.FP64 else np.float32
    return [np.asarray(w.u0, dt) for w in ws]


@pytest.mark.parametrize("prec", [B.FP64, B.FP32])
def test_euler_batch_matches_single_and_oracle(prec):
    _say(f"euler batch prec={prec}")
    ws = I.euler_riemann_batch(count=10, seed=3, nmin=256, nmax=900)
    ws[3] = ws[3].with_(bc=I.PERIODIC)  # per-instance parameters may differ
    ws[5] = ws[5].with_(cfl=0.3)
    T = [0.2 - 0.01 * b for b in range(len(ws))]
    states = _states(ws, prec)
    with B.Batch(states, [B.workload_params(w, prec) for w in ws]) as bt:
        stats, rc = bt.solve(T)
        got = [bt.read(b) for b in range(len(ws))]
    assert rc == B.OK
    for b, w in enumerate(ws):
        check_sums(stats[b], got[b], 3, w.dx)
        with B.Solver(states[b], **B.workload_params(w, prec)) as s:
            st = s.solve(T[b])
            alone = s.read()
        assert st["nsteps"] == stats[b]["nsteps"] and st["t"] == stats[b]["t"]
        assert np.array_equal(alone, got[b]), b
        if prec == B.FP64:
            uo, to, no = O.solve(_oracle_problem(w), w.u0, T[b])
            assert no == stats[b]["nsteps"]
            assert np.max(np.abs(got[b] - uo)) <= 1e-12


def test_scalar_batch_with_ragged_sizes_fp64():
    _say("scalar batch ragged")
    rng = np.random.default_rng(4)
    ws = []
    for b, n in enumerate([1, 7, 253, 254, 255, 509, 1000]):
        u0 = 0.5 + I.sine_cell_averages(n) + 0.1 * rng.uniform(-1, 1, n)
        ws.append(I.Workload(name=f"s{b}", nx=n, flux=I.BURGERS, u0=u0, T=0.3,
                             bc=I.PERIODIC if b % 2 else I.TRANSMISSIVE))
    with B.Batch(_states(ws, B.FP64), [B.workload_params(w) for w in ws]) as bt:
        stats, rc = bt.solve(0.3)
        for b, w in enumerate(ws):
            uo, _, no = O.solve(_oracle_problem(w), w.u0, 0.3)
            assert stats[b]["nsteps"] == no
            assert np.array_equal(bt.read(b), uo), b


def test_batch_error_is_isolated():
    _say("batch error isolation")
    ws = I.euler_riemann_batch(count=4, seed=9, nmin=300, nmax=400)
    bad = I.burgers_noisy(n=300, seed=1, cfl=40.0, T=1000.0)
    ws2 = [I.burgers_noisy(n=300 + 10 * b, seed=b) for b in range(3)] + [bad]
    with B.Batch(_states(ws2, B.FP64), [B.workload_params(w) for w in ws2]) as bt:
        stats, rc = bt.solve([w.T for w in ws2], raise_on_error=False)
        assert rc == B.ENONFINITE
        assert stats[3]["err"] == B.ENONFINITE
        for b in range(3):
            assert stats[b]["err"] == 0
            uo, to, _ = O.solve(_oracle_problem(ws2[b]), ws2[b].u0, ws2[b].T)
            assert np.array_equal(bt.read(b), uo)
        u_bad = bt.read(3)
        assert np.all(np.isfinite(u_bad))
    del ws


def test_batch_second_solve_continues():
    _say("batch resume")
    ws = [I.burgers_noisy(n=400 + 37 * b, seed=b) for b in range(5)]
    with B.Batch(_states(ws, B.FP64), [B.workload_params(w) for w in ws]) as bt:
        bt.solve([0.05 * (b + 1) for b in range(5)])  # instances stop at different steps
        bt.solve(0.3)
        for b, w in enumerate(ws):
            uo, t1, _ = O.solve(_oracle_problem(w), w.u0, 0.05 * (b + 1))
            uo, _, _ = O.solve(_oracle_problem(w), uo, 0.3, t=t1)
            assert np.array_equal(bt.read(b), uo), b


def test_full_size_riemann_batch_sampled_fp32():
    """The 4096-instance Riemann batch in the benchmark's form (float bulk, one launch per stage,
    autotuned block), 25 steps: sampled instances agree with the FP64 oracle on their float
    inputs and with their own solo solves bit for bit."""
    _say("full-size riemann batch fp32 (4096 instances)")
    ws = I.euler_riemann_batch(count=4096, seed=3)
    states = _states(ws, B.FP32)
    T = [w.T for w in ws]
    with B.Batch(states, [B.workload_params(w, B.FP32) for w in ws]) as bt:
        stats, rc = bt.solve(T, 25)
        assert rc == B.OK
        picks = [0, 1, 777, 2048, 3001, 4095]
        got = {b: bt.read(b) for b in picks}
    for b in picks:
        w = ws[b]
        assert stats[b]["nsteps"] == 25
        uo, _, _ = O.solve(_oracle_problem(w), states[b].astype(np.float64), w.T, max_steps=25)
        # Riemann data: the jump makes a few cells sensitive to rounding (L1 bound, as for Sod)
        assert np.mean(np.abs(got[b] - uo)) <= 1e-4, b
        # element-wise 1e-5 (relative above 1) away from the waves
        assert_fp32_close(got[b], uo, 3, smooth_cells(uo, 3, (w.nx,)))
        check_sums(stats[b], got[b], 3, w.dx)
        with B.Solver(states[b], **B.workload_params(w, B.FP32)) as s:
            s.solve(w.T, 25)
            assert np.array_equal(s.read(), got[b]), b


@pytest.mark.parametrize("prec", [B.FP64, B.FP32])
def test_large_instances_spread_their_alpha(prec, monkeypatch):
    """A batch holding instances of more than 128 tiles runs the kernel that spreads an instance's
    alpha over entries (small instances of the same launch keep their own slot): every instance
    equals its solve alone bit for bit, and the double bulk the oracle."""
    _say(f"batch of large instances prec={prec}")
    monkeypatch.setenv("NPW_BLOCK", "64")
    ws = [I.burgers_noisy(n=n, seed=s, T=0.05) for n, s in ((70001, 1), (200, 2), (20000, 3))]
    states = _states(ws, prec)
    with B.Batch(states, [B.workload_params(w, prec) for w in ws]) as bt:
        stats, rc = bt.solve([w.T for w in ws], 8)
        got = [bt.read(b) for b in range(len(ws))]
    assert rc == B.OK
    for b, w in enumerate(ws):
        assert stats[b]["nsteps"] == 8
        with B.Solver(states[b], **B.workload_params(w, prec)) as s:
            st = s.solve(w.T, max_steps=8)
            alone = s.read()
        assert st["t"] == stats[b]["t"] and st["alpha"][0] == stats[b]["alpha"][0]
        assert np.array_equal(alone, got[b]), b
        if prec == B.FP64:
            uo, to, _ = O.solve(_oracle_problem(w), w.u0, w.T, max_steps=8)
            assert np.array_equal(got[b], uo) and to == stats[b]["t"]
