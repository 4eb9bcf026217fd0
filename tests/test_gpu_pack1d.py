"""GPU tests of the packed alpha slots of 1D single grids (one entry per tile, written with a plain
store and read whole by the next stage; grids of at most 1280 tiles at 64 or 128 threads per
workgroup) against the FP64 oracle and against the spread entries that larger grids and 256- and
512-thread launches keep.  Global Lax-Friedrichs takes alpha as the maximum wave speed over the
whole grid (Section 7), so however the maximum is gathered the steps must be the oracle's bit for
bit in double, and the same bits in float on either path."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1602_00182_amd import binding as B
from paper_1602_00182_amd import inputs as I

pytestmark = pytest.mark.gpu

PACK_MAX = 1280  # tiles a packed slot holds


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _problem(w):
    return O.Problem(nx=w.nx, flux=w.flux, dim=w.dim, ny=w.ny, ncomp=w.ncomp, bc=w.bc, x0=w.x0, x1=w.x1,
                     speed_x=w.speed_x, gamma=w.gamma, cfl=w.cfl, eps_weno=w.eps_weno, eps_m=w.eps_m,
                     recon=w.recon, switch_mode=w.switch_mode, dt_fixed=w.dt_fixed)


def _burgers(n, seed, amp=1.0):
    """Smooth data plus sparse jumps, so that alpha comes from a few cells somewhere in the grid."""
    rng = np.random.default_rng(seed)
    u = 0.5 + amp * I.sine_cell_averages(n) + 0.3 * rng.uniform(-1, 1, n) * (rng.random(n) < 0.05)
    return I.Workload(name="pack", nx=n, flux=I.BURGERS, u0=u, T=1.0, bc=I.PERIODIC)


@pytest.mark.parametrize("block,tiles", [(64, PACK_MAX), (64, PACK_MAX + 1), (128, PACK_MAX), (128, PACK_MAX + 1),
                                         (64, 1), (64, 2), (128, 3)])
def test_tile_counts_around_the_packed_limit_fp64(block, tiles, monkeypatch):
    """Grids of exactly the largest packed tile count and one tile more (spread entries), and of
    one to three tiles, whose alpha cell sits in the last tile: steps bit for bit."""
    n = (block - 2) * (tiles - 1) + 5
    _say(f"pack limit block={block} tiles={tiles} n={n}")
    monkeypatch.setenv("NPW_BLOCK", str(block))
    w = _burgers(n, 3)
    u0 = w.u0.copy()
    u0[n - 2] = 2.5  # the largest wave speed, in the last tile
    w = w.with_(u0=u0)
    with B.Solver(w.u0, **B.workload_params(w)) as s:
        assert s.launch_shape()["block"] == block
        L = s.rhs()
        st = s.solve(w.T, max_steps=4)
        u = s.read()
    Lo, _ = O.rhs(_problem(w), w.u0)
    assert np.array_equal(L, Lo)
    uo, to, no = O.solve(_problem(w), w.u0, w.T, max_steps=4)
    assert st["nsteps"] == no == 4 and st["t"] == to
    assert np.array_equal(u, uo)


def test_float_packed_and_spread_paths_agree_bitwise(monkeypatch):
    """The same float grid at 64 threads (packed entries) and at 256 threads (spread entries):
    every cell is computed with the same arithmetic and alpha is an exact maximum, so the states
    after 40 steps are equal bit for bit."""
    _say("pack vs spread fp32")
    w = _burgers(20000, 5)
    u32 = np.asarray(w.u0, np.float32)
    out = {}
    for block in ("64", "256"):
        monkeypatch.setenv("NPW_BLOCK", block)
        with B.Solver(u32, **B.workload_params(w, B.FP32)) as s:
            st = s.solve(w.T, max_steps=40)
            out[block] = (s.read(), st["t"], st["alpha"][0])
    assert np.array_equal(out["64"][0], out["256"][0])
    assert out["64"][1:] == out["256"][1:]


@pytest.mark.parametrize("prec", [B.FP64, B.FP32])
def test_replaced_state_takes_its_own_alpha(prec, monkeypatch):
    """Solve a state with a large wave speed, then write one with a smaller one into the same
    solver: the state check clears the packed slots, so the next steps use the new state's alpha
    and equal a fresh solver's bit for bit."""
    _say(f"pack state replacement prec={prec}")
    monkeypatch.setenv("NPW_BLOCK", "64")
    big = _burgers(9000, 7, amp=2.0)
    small = _burgers(9000, 8, amp=0.3)
    cast = (lambda u: np.asarray(u, np.float32)) if prec == B.FP32 else (lambda u: u)
    with B.Solver(cast(big.u0), **B.workload_params(big, prec)) as s:
        s.solve(big.T, max_steps=25)
        s.write(cast(small.u0), 0.0)
        st = s.solve(small.T, max_steps=6)
        got = s.read()
    with B.Solver(cast(small.u0), **B.workload_params(small, prec)) as s:
        st2 = s.solve(small.T, max_steps=6)
        ref = s.read()
    assert np.array_equal(got, ref) and st["t"] == st2["t"]
    if prec == B.FP64:
        uo, to, _ = O.solve(_problem(small), small.u0, small.T, max_steps=6)
        assert np.array_equal(got, uo) and st["t"] == to


def test_error_then_new_state_on_packed_slots(monkeypatch):
    """A solve that blows up keeps its last good step (the oracle's); a state written into the
    same solver afterwards steps as the oracle does (one step clipped to a short T, so alpha acts
    through the flux only): no entry of the failed stage survives the state check."""
    _say("pack blowup then new state")
    monkeypatch.setenv("NPW_BLOCK", "64")
    w = I.burgers_noisy(n=4000, seed=1, cfl=40.0, T=1000.0)
    fresh = _burgers(4000, 9).u0
    with B.Solver(w.u0, **B.workload_params(w)) as s:
        with pytest.raises(B.NpwError) as e:
            s.solve(w.T)
        assert e.value.code == B.ENONFINITE
        n_good = s.stats()["nsteps"]
        u = s.read()
        uo, _, _ = O.solve(_problem(w), w.u0, w.T, max_steps=n_good)
        assert np.array_equal(u, uo)
        s.write(fresh, 0.0)
        st = s.solve(1e-4)
        got = s.read()
    uo, to, no = O.solve(_problem(w), fresh, 1e-4)
    assert st["nsteps"] == no == 1 and st["t"] == to
    assert np.array_equal(got, uo)
