"""Benchmark: cell-updates/s per RK stage of the non-polynomial WENO5 solver on one MI355X.

Workload (default): 1D Burgers u_t + (u^2/2)_x = 0, periodic on [-1, 1], N = 65536 cells,
u0 = 0.5 + sin(pi x) + seeded U(-1e-3, 1e-3) noise, global Lax-Friedrichs, SSP-RK3 at CFL 0.5
to T = 1.5/pi (past shock formation, ~47k steps), RBF-WENO5 with the monotone switch.
One benchmark "step" = one whole solve from the initial state (state reset from a resident
device copy, not timed as host traffic).  value = N * 3 * (RK steps) * solves / seconds.

Prints one JSON line.  Only one GPU is supported; --gpus N > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per cell and RK stage for a scalar state: stage 1 reads u^n and writes
# u^(1); stages 2 and 3 read u^n, read the stage input and write the output -> (2 + 3 + 3) / 3
# element accesses per cell-stage.
ELEM_ACCESSES_PER_CELL_STAGE = 8.0 / 3.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed whole solves")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: only one GPU is supported by this build (asked for {max(args.gpus, world)})",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1602_00182_amd import binding as B
    from paper_1602_00182_amd import inputs as I

    torch.cuda.set_device(0)
    prec = B.FP32 if args.precision == "fp32" else B.FP64
    tdt = torch.float32 if prec == B.FP32 else torch.float64
    w = I.burgers_noisy(n=args.n, seed=2)
    u0_dev = torch.tensor(w.u0, dtype=tdt, device="cuda")
    stream = torch.cuda.Stream()  # default priority
    solver = B.Solver(u0_dev, stream=stream.cuda_stream, **B.workload_params(w, prec))

    def one_solve():
        solver.write(u0_dev, 0.0)
        st = solver.solve(w.T)
        return st

    for _ in range(args.warmup):
        one_solve()
    torch.cuda.synchronize()
    lat = []
    nsteps = None
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        a = time.perf_counter()
        st = one_solve()
        lat.append(time.perf_counter() - a)
        nsteps = st["nsteps"]
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)

    cell_stages = float(w.nx) * 3.0 * nsteps * args.steps
    value = cell_stages / wall
    esize = 4 if prec == B.FP32 else 8
    launches = 3 * nsteps * args.steps
    avg_launch_s = (gpu_ms / 1e3) / launches
    bytes_per_launch = ELEM_ACCESSES_PER_CELL_STAGE * esize * w.nx
    achieved = bytes_per_launch / avg_launch_s / 1e9

    out = {
        "metric": "cell-updates/s per RK stage (1D Burgers N=65536, RBF-WENO5 + monotone switch, "
                  "global LF, SSP-RK3 CFL 0.5 to T=1.5/pi)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == B.FP32 else "f64",
        "data": "synthetic (seeded)",
        "config": {"workload": "burgers_noisy_N65536", "N": w.nx, "T": w.T, "cfl": w.cfl,
                   "rk_steps_per_solve": nsteps, "eta_precision": "f64"},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "stage1d_kernel", "avg_launch_us": avg_launch_s * 1e6},
    }

    if not args.no_cpu_baseline:
        import oracle as O
        pb = O.Problem(nx=w.nx, flux=w.flux, cfl=w.cfl, eps_weno=w.eps_weno, eps_m=w.eps_m,
                       recon=w.recon, switch_mode=w.switch_mode)
        u_ref = np.asarray(w.u0, np.float32 if prec == B.FP32 else np.float64).astype(np.float64)
        # size the sample to the time budget from one timed step
        a = time.perf_counter()
        u1, t1, _ = O.step(pb, u_ref, w.T)
        per_step = time.perf_counter() - a
        k = max(1, int(args.cpu_seconds / max(per_step, 1e-6)))
        a = time.perf_counter()
        uo, to, no = O.solve(pb, u1, w.T, t=t1, max_steps=k - 1)
        el = time.perf_counter() - a + per_step
        ksteps = no + 1
        out["cpu_baseline"] = {"value": w.nx * 3.0 * ksteps / el, "unit": "cell-updates/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"first {ksteps} RK3 steps of the same N={w.nx} solve, FP64, one thread"}
        solver.write(u0_dev, 0.0)
        solver.solve(w.T, max_steps=ksteps)
        ug = solver.read().astype(np.float64)
        out["l1_vs_oracle"] = {"steps": ksteps, "l1": float(np.mean(np.abs(ug - uo))),
                               "linf": float(np.max(np.abs(ug - uo)))}
    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
