"""Serving loop (continuous batching): requests admitted as slots and HBM free up, stepped
together, and each result identical to the same solve run alone."""
import sys

import numpy as np
import pytest

import oracle as O
from conftest import check_sums
from paper_1602_00182_amd import binding as B
from paper_1602_00182_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _requests(count, seed, nmax, tmax):
    reqs = I.serving_trace(nreq=count, seed=seed, nmax=nmax)
    return [r.work.with_(T=min(r.work.T, tmax)) for r in reqs]


def _drain(srv, ids, max_pumps=20000, steps=16):
    saw_queue = False
    for _ in range(max_pumps):
        nr, nq = srv.pump(steps)
        saw_queue |= nq > 0 and nr > 0
        if nr == 0 and nq == 0:
            return saw_queue
    raise AssertionError("serving loop did not drain")


@pytest.mark.parametrize("prec", [B.FP32, B.FP64])
def test_results_identical_alone_and_in_the_mix(prec):
    _say(f"serving mix prec={prec}")
    ws = _requests(14, seed=4, nmax=6000, tmax=0.15)
    esize = 4 if prec == B.FP32 else 8
    budget = 3 * esize * 24000  # the arena holds 24k elements: a few requests at a time (Euler N=6000 is 18k)
    with B.Server(budget, max_slots=3, precision=prec) as srv:
        ids = [srv.submit(w.u0, w.T, **B.workload_params(w, prec)) for w in ws]
        saw_queue = _drain(srv, ids)
        assert saw_queue
        for rid, w in zip(ids, ws):
            out, st, rc = srv.poll(rid)
            assert rc == B.OK
            dt = np.float32 if prec == B.FP32 else np.float64
            with B.Solver(np.asarray(w.u0, dt), **B.workload_params(w, prec)) as s:
                st1 = s.solve(w.T)
                alone = s.read()
            assert st["nsteps"] == st1["nsteps"]
            assert np.array_equal(out, alone), rid
            # the reported sums are those of the final state, as for the solo solve
            check_sums(st, out, w.ncomp, w.dx)
            assert st["mass"] == st1["mass"] and st["alpha"][0] == st1["alpha"][0]
            if prec == B.FP64 and w.nx <= 2000:
                pb = O.Problem(nx=w.nx, flux=w.flux, ncomp=w.ncomp, bc=w.bc, cfl=w.cfl, gamma=w.gamma)
                uo, _, _ = O.solve(pb, w.u0, w.T)
                assert np.array_equal(out, uo)
            a, b, c = srv.times(rid)
            assert a <= b <= c


@pytest.mark.parametrize("prec", [B.FP32, B.FP64])
def test_large_request_spreads_its_alpha(prec):
    """A request of more than 128 tiles of the pools' 512-thread workgroups spreads its alpha over
    entries; served beside small ones it still equals its solve alone bit for bit."""
    _say(f"serving large request prec={prec}")
    ws = [I.burgers_noisy(n=n, seed=s, T=0.02) for n, s in ((70001, 5), (300, 6), (1500, 7))]
    esize = 4 if prec == B.FP32 else 8
    with B.Server(3 * esize * 80000, max_slots=4, precision=prec) as srv:
        ids = [srv.submit(w.u0, w.T, **B.workload_params(w, prec)) for w in ws]
        _drain(srv, ids)
        dt = np.float32 if prec == B.FP32 else np.float64
        for rid, w in zip(ids, ws):
            out, st, rc = srv.poll(rid)
            assert rc == B.OK
            with B.Solver(np.asarray(w.u0, dt), **B.workload_params(w, prec)) as s:
                st1 = s.solve(w.T)
                alone = s.read()
            assert st["nsteps"] == st1["nsteps"] and np.array_equal(out, alone), rid


def test_failing_request_does_not_poison_others():
    _say("serving failure isolation")
    good = _requests(5, seed=7, nmax=3000, tmax=0.1)
    bad = I.burgers_noisy(n=500, seed=1, cfl=40.0, T=1000.0)
    with B.Server(64 << 20, max_slots=8, precision=B.FP64) as srv:
        ids = [srv.submit(w.u0, w.T, **B.workload_params(w)) for w in good]
        bad_id = srv.submit(bad.u0, bad.T, **B.workload_params(bad))
        _drain(srv, ids + [bad_id])
        out, st, rc = srv.poll(bad_id)
        assert rc == B.ENONFINITE and np.all(np.isfinite(out))
        check_sums(st, out, 1, bad.dx)  # the sums of the last good state it returns
        for rid, w in zip(ids, good):
            out, st, rc = srv.poll(rid)
            assert rc == B.OK
            with B.Solver(w.u0, **B.workload_params(w)) as s:
                s.solve(w.T)
                assert np.array_equal(out, s.read())


def test_submit_validation():
    _say("serving validation")
    with B.Server(1 << 20, max_slots=2, precision=B.FP32) as srv:
        w = I.advection_sine(100)
        with pytest.raises(B.NpwError):
            srv.submit(w.u0, 1.0, **B.workload_params(w, B.FP64))  # precision mismatch
        with pytest.raises(B.NpwError):
            big = np.zeros(200000)
            srv.submit(big, 1.0, nx=200000, flux=B.BURGERS, precision=B.FP32)  # can never fit


def test_pump_advances_exactly_the_requested_steps():
    """pump(7) is a 4-step graph and three 1-step graphs (each flips the ping-pong buffer);
    requests admitted after odd pumps must start from the right buffer."""
    _say("serving pump step count")
    d = 2.0 ** -10  # binary dt, so t sums exactly to the step count
    w = I.advection_sine(64, dt_fixed=d)
    prm = B.workload_params(w)
    with B.Server(1 << 20, max_slots=4, precision=B.FP64) as srv:
        a = srv.submit(w.u0, 6 * d, **prm)
        b = srv.submit(w.u0, 13 * d, **prm)
        srv.pump(7)
        assert srv.poll(a) is not None and srv.poll(b) is None
        c = srv.submit(w.u0, 3 * d, **prm)  # admitted with u^n in the other buffer
        srv.pump(5)
        assert srv.poll(b) is None and srv.poll(c) is not None
        srv.pump(1)
        for rid, n in ((a, 6), (b, 13), (c, 3)):
            out, st, rc = srv.poll(rid)
            assert rc == B.OK and st["nsteps"] == n
            with B.Solver(w.u0, **prm) as s:
                s.solve(n * d)
                assert np.array_equal(out, s.read()), rid
