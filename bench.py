"""Benchmark of the non-polynomial WENO5 solver on one MI355X.

Default workload (the headline, the largest single-GPU configuration): 2D Euler dimension by
dimension (Section 7, eq. 2DIntegral, one midpoint point per face) on 2048 x 2048 cells of
[0,1]^2, four seeded constant quadrant states split at (0.5, 0.5), transmissive, gamma = 1.4,
SSP-RK3 at CFL 0.4 to T = 0.25 (about 10^4 RK steps), RBF-WENO5 with the monotone switch, float
bulk with double eta/switch.  One benchmark "step" is one whole solve from the initial state (the
state is reset from a resident device copy).
value = cells * 3 stages * RK steps * solves / wall seconds (cell-updates per RK stage).

Other workloads (--workload): burgers (1D Burgers N = 65536, 0.5 + sin(pi x) + seeded noise, to
T = 1.5/pi), euler_batch (4096 Riemann problems, N in [256, 4096], to T = 0.2), serving (a Poisson
trace through the continuous-batching loop, compared with one solve at a time), advection (sin(pi x)
at N = 65536 to T = 0.5) and advection2d (sin(2 pi (x + y)) on 2048^2 to T = 0.25), the paper's
smooth test problems at the headline's sizes, on which the k = 2 and Section 6 reconstructions are
defined everywhere (their shape parameter is singular where a solution with non-zero curvature
crosses zero).  --recon and --variables pick the reconstruction.

Prints one JSON line.  Only one GPU: --gpus N > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed-FP32 instructions (which this build disables): 256 CUs x 4 SIMDs
# x 16 lanes x 2 flops per FMA x 2.4 GHz.  The published 157.3 TFLOP/s counts packed FMAs.
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Algorithmic FP32 flops of one scalar reconstruction + flux + update along one direction, per cell
# and RK stage (smoothness indicators 21, substencil values 42, weights ~30, combination 6, LF flux
# ~8, update ~5, switch ~8), and the Euler equation of state per cell and direction (~30, one sqrt).
FLOPS_SCALAR_SWEEP = 130.0
FLOPS_EULER_EOS = 30.0
# Algorithmic HBM element accesses per cell, component and RK stage: stage 1 reads u^n and
# writes u^(1); stages 2 and 3 read u^n and the stage input and write the output.
ACCESSES_PER_CELL_STAGE = 8.0 / 3.0
METRIC = "cell-updates/s per RK stage at stated L1 err vs FP64 oracle; p50/p99 solve latency"


KERNEL_SOURCES = ("npw_device.h", "npw_internal.h", "npw_kernels.h", "npw_kernels2d.h", "npw_kernels2d_strip.h",
                  "npw_kernels_f32.hip", "npw_kernels_f64.hip")

# reconstruction codes of include/npweno.h by name
RECONS = {"rbf_weno5": 0, "weno5_js": 1, "rbf_eno3": 2, "eno3": 3, "rbf_weno3": 4, "weno3_js": 5, "rbf_eno2": 6,
          "eno2": 7, "rbf_eno2_2d": 8}
FLUX_NAMES = {0: "Advection", 1: "Burgers", 2: "Euler"}


def kernel_label(w, prec, shape, batched=False):
    """Name of the stage-kernel instantiation a workload runs (the key of the counter summaries):
    template arguments as in the source, plus k2 (compiled with the k = 2 code) and char
    (characteristic-wise) when they apply."""
    R = "float" if prec == 1 else "double"
    extra = (", k2" if w.recon >= 4 else "") + (", char" if w.variables == 1 else "")
    if w.dim == 1:
        lab = f"stage1d_kernel<{R}, {FLUX_NAMES[w.flux]}, {w.ncomp}, {shape['block']}{extra}>"
        return lab + " (batched)" if batched else lab
    if shape["tile_y"] > 8:  # a column strip walked 4 rows at a time
        return f"stage2d_strip_kernel<{R}, {FLUX_NAMES[w.flux]}, {w.ncomp}, {shape['tile_x']}, {shape['tile_y']}>"
    share = "" if shape["lds_shared"] else ", recompute"
    return f"stage2d_kernel<{R}, {FLUX_NAMES[w.flux]}, {w.ncomp}, {shape['tile_x']}, {shape['tile_y']}{share}{extra}>"


def scheme_of(w):
    name = {v: k for k, v in RECONS.items()}[w.recon]
    return (name + (", characteristic" if w.variables == 1 else "")
            + (", monotone switch off" if w.switch_mode == 1 else ", monotone switch"))


def kernel_source_hash() -> str:
    """Short hash of the stage-kernel sources; a counter summary stays valid while it matches."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1602_00182_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the FETCH_SIZE/WRITE_SIZE summaries under profiles/
    (each counter scaled by what it reads for a copy of known size), or None when no summary
    covers this kernel as it is now built."""
    key = "kernel=" + kernel.replace(" ", "")
    src = "source=" + kernel_source_hash()
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    for name in sorted(os.listdir(pdir)):
        if not name.endswith("_hbm_counters.txt"):
            continue
        with open(os.path.join(pdir, name)) as f:
            for line in f:
                parts = line.split()
                if parts and parts[0] == "traffic" and key in parts and src in parts:
                    return float(next(p for p in parts if p.startswith("bytes_per_launch="))[len("bytes_per_launch="):])
    return None


def counter_valu(kernel: str):
    """VALU wave-instructions per launch of `kernel` and their split into instruction classes, from
    the VALU counter summaries under profiles/, or None when none covers this kernel as now built."""
    key = "kernel=" + kernel.replace(" ", "")
    src = "source=" + kernel_source_hash()
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    for name in sorted(os.listdir(pdir)):
        if not name.endswith("_valu_counters.txt"):
            continue
        with open(os.path.join(pdir, name)) as f:
            for line in f:
                parts = line.split()
                if parts and parts[0] == "valu" and key in parts and src in parts:
                    kv = dict(p.split("=", 1) for p in parts[1:] if "=" in p)
                    if "classes" not in kv:
                        return None
                    classes = {c: float(v) for c, v in (x.split(":") for x in kv["classes"].split(","))}
                    return {"wave_instr_per_launch": float(kv["wave_instr_per_launch"]),
                            "wave_instr_per_cell_stage": float(kv["wave_instr_per_cell_stage"]),
                            "classes": classes, "summary": name}
    return None


# The counters split compares, selects, moves and bit logic into no classes of their own; the probe
# replays that remainder in the proportions of the 2D Euler stage's code (compares 6, selects 8,
# moves 4, logic 3).
REST_SPLIT = {"cmp": 6.0, "cnd": 8.0, "mov": 4.0, "logic": 3.0}
_CEILINGS = {}


def probe_argv(classes: dict) -> list:
    """valu_mix_probe arguments for counted instruction classes (the remainder split by REST_SPLIT)."""
    mix = {k: v for k, v in classes.items() if k != "rest"}
    rest = classes.get("rest", 0.0)
    tot = sum(REST_SPLIT.values())
    for k, w in REST_SPLIT.items():
        mix[k] = mix.get(k, 0.0) + rest * w / tot
    return [f"{k}={v:.3f}" for k, v in sorted(mix.items()) if v > 0]


def valu_ceiling(classes: dict):
    """Wave-instructions per second that the whole GPU sustains on this instruction mix, measured
    by the valu_mix_probe program (built beside the library), or None if it cannot run."""
    import subprocess
    argv = probe_argv(classes)
    key = " ".join(argv)
    if key not in _CEILINGS:
        exe = os.path.join(ROOT, "paper_1602_00182_amd", "valu_mix_probe")
        try:
            r = subprocess.run([exe, *argv], capture_output=True, text=True, timeout=120)
            _CEILINGS[key] = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None
            if r.returncode != 0:
                progress(f"valu_mix_probe failed ({r.returncode}): {r.stderr.strip()[-200:]}")
        except (OSError, subprocess.TimeoutExpired, ValueError, IndexError) as e:
            progress(f"valu_mix_probe did not run: {e}")
            _CEILINGS[key] = None
    return _CEILINGS[key]


def valu_roof(label: str, avg_launch: float = None, cell_stages_per_s: float = None):
    """Issue rate of the kernel's VALU instructions against the ceiling of its own mix.  The counters
    give the instructions of one launch (and per cell-stage); this run's event timing gives the rate:
    per launch over the average launch, or per cell-stage times the cell-stages done per second
    (batches, whose launches narrow as instances finish)."""
    c = counter_valu(label)
    if c is None:
        return None
    ceil = valu_ceiling(c["classes"])
    if cell_stages_per_s is not None:
        rate = c["wave_instr_per_cell_stage"] * cell_stages_per_s
    else:
        rate = c["wave_instr_per_launch"] / avg_launch
    out = {"issue_rate": rate, "unit": "wave-instructions/s", "wave_instr_per_launch": c["wave_instr_per_launch"],
           "wave_instr_per_cell_stage": c["wave_instr_per_cell_stage"], "counters": c["summary"]}
    if ceil is not None:
        out.update({"ceiling": ceil["wave_instr_per_s"], "frac": rate / ceil["wave_instr_per_s"],
                    "ceiling_mix_per_200": ceil["mix_per_round"],
                    "ceiling_basis": "valu_mix_probe: the kernel's counted VALU mix replayed with no memory "
                                     "traffic or dependency stalls, best of 8/6/4 register chains"})
    return out


def alg_flops_per_cell_stage(w) -> float:
    """Algorithmic FP32 flops per cell and RK stage: every component reconstructed along every
    direction, plus the equation of state per direction for Euler."""
    per_dir = w.ncomp * FLOPS_SCALAR_SWEEP + (FLOPS_EULER_EOS if w.flux == 2 else 0.0)
    return w.dim * per_dir


def host_description() -> dict:
    """Host CPU model and core counts (the oracle baseline runs on these cores)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed whole solves (default: 20 for burgers and advection, so p50/p99 rest on 20 "
                         "samples; 3 for euler2d and advection2d; 2 for euler_batch)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["burgers", "advection", "euler2d", "advection2d", "euler_batch", "serving"],
                    default="euler2d")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--n", type=int, default=None, help="override the grid size")
    ap.add_argument("--max-rk-steps", type=int, default=-1,
                    help="stop each solve after this many RK steps (profiling runs only; not a bench value)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle sample")
    ap.add_argument("--cpu-workers", type=int, default=None,
                    help="oracle processes of the all-core baseline (default: the host cores, at most 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error-at-t", action="store_true",
                    help="skip the double-bulk GPU solve that gives the float error at T (2D workloads)")
    ap.add_argument("--oracle-sample", default=None, help=argparse.SUPPRESS)  # worker mode of the CPU baseline
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--recon", choices=sorted(RECONS), default=None,
                    help="reconstruction (default: each workload's own, rbf_weno5 with the monotone switch)")
    ap.add_argument("--variables", choices=["componentwise", "characteristic"], default="componentwise",
                    help="Euler reconstruction variables (euler_batch and euler2d)")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-nmax", type=int, default=262144,
                    help="upper end of the request grid sizes: N is drawn log-uniform in [256, nmax]")
    ap.add_argument("--serving-tscale", type=float, default=0.02,
                    help="factor on every request's T (drawn in [0.1, 1]) so that the trace's work fits a run")
    ap.add_argument("--serving-budget-mib", type=float, default=64.0,
                    help="HBM arena of the server (small enough that admission binds)")
    ap.add_argument("--serving-solo", type=int, default=200,
                    help="requests (from the start of the trace) also solved one at a time for comparison")
    ap.add_argument("--pump-steps", type=int, default=64, help="RK steps per serving pump (admission granularity)")
    return ap.parse_args()


def progress(msg: str) -> None:
    """One line on stderr per finished piece of work (a solve, a baseline leg), so a long run shows
    that it is moving; the result stays the single JSON line on stdout."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _percentiles(x):
    return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99))}


def _time_solves(solver, reset, T, steps, warmup, max_rk, stream):
    """Wall time of `steps` reset+solve rounds, plus the GPU time of the solves alone: a pair of
    events on the solver's stream brackets each solve(), so the state reset is not counted."""
    import torch
    for i in range(warmup):
        reset()
        solver.solve(T, max_rk)
        progress(f"warmup solve {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    lat = []
    evs = []
    t0 = time.perf_counter()
    rk = 0
    for i in range(steps):
        a = time.perf_counter()
        reset()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st = solver.solve(T, max_rk)
        e1.record(stream)
        evs.append((e0, e1))
        lat.append(time.perf_counter() - a)
        rk = st["nsteps"]
        progress(f"timed solve {i + 1}/{steps}: {lat[-1]:.3f} s, {rk} RK steps")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = sum(e0.elapsed_time(e1) for e0, e1 in evs) / 1e3
    return wall, gpu_s, lat, rk


def apply_scheme(args, w):
    """The workload with the reconstruction and variables asked for on the command line."""
    kw = {}
    if args.recon is not None:
        kw["recon"] = RECONS[args.recon]
    if args.variables == "characteristic":
        if w.flux != 2:
            raise SystemExit("bench.py: --variables characteristic needs an Euler workload")
        kw["variables"] = 1
    return w.with_(**kw) if kw else w


def bench_single(args, w, prec):
    """A single grid (1D or 2D) solved from its initial state `steps` times."""
    import torch

    from paper_1602_00182_amd import binding as B
    tdt = torch.float32 if prec == B.FP32 else torch.float64
    u0_dev = torch.tensor(w.u0, dtype=tdt, device="cuda")
    stream = torch.cuda.Stream()
    solver = B.Solver(u0_dev, stream=stream.cuda_stream, **B.workload_params(w, prec))
    shape = solver.launch_shape()
    progress(f"solver created ({w.name}, launch shape {shape})")
    label = kernel_label(w, prec, shape)
    wall, gpu_s, lat, rk = _time_solves(solver, lambda: solver.write(u0_dev, 0.0), w.T, args.steps, args.warmup,
                                        args.max_rk_steps, stream)
    u_T = solver.read()  # the state at T of the last timed solve (float error at T below)
    ncell = w.ncell
    cell_stages = float(ncell) * 3.0 * rk * args.steps
    esize = 4 if prec == B.FP32 else 8
    launches = 3 * rk * args.steps
    avg_launch = gpu_s / launches
    out = {
        "value": cell_stages / wall,
        "ms_per_step": 1e3 * wall / args.steps,
        "latency_s": _percentiles(lat),
        "rk_steps_per_solve": rk,
        "roofline": roofline(w, label, ncell, esize, avg_launch),
        "launch_shape": shape,
        "u_T": u_T,
    }
    return out, solver, u0_dev


def roofline(w, label, cells_per_launch, esize, avg_launch, traffic=None):
    """Roofline of the dominant kernel (the fused RK stage) from its event-timed average launch.
    2D and Euler stages are bound by VALU arithmetic (their issue utilisation is at the chip's
    limit), so they report an ALU roofline with the HBM fraction beside it; the 1D scalar stages
    report HBM (they are latency-bound, far below either roof)."""
    bytes_per_launch = ACCESSES_PER_CELL_STAGE * esize * w.ncomp * cells_per_launch
    gbs = bytes_per_launch / avg_launch / 1e9
    flops = alg_flops_per_cell_stage(w) * cells_per_launch
    tflops = flops / avg_launch / 1e12
    if traffic is None:
        traffic = counter_traffic(label)
    hbm = {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
           "bytes_per_launch": bytes_per_launch}
    alu = {"achieved": tflops, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tflops / ALU_PEAK_TFLOPS,
           "flops_per_launch": flops, "flops_per_cell_stage": alg_flops_per_cell_stage(w)}
    common = {"traffic": traffic, "valu": valu_roof(label, avg_launch), "kernel": label,
              "avg_launch_us": avg_launch * 1e6}
    if w.dim == 2 or w.flux == 2:
        return {"bound": "alu", **{k: alu[k] for k in ("achieved", "peak", "unit", "frac")}, **common,
                "limiter": "VALU issue: see valu.frac, the issue rate against the ceiling of the kernel's own "
                           "instruction mix",
                "flops_per_launch": flops, "peak_basis": "FP32 vector FMA without packed-FP32 instructions",
                "hbm": hbm}
    return {"bound": "hbm", **{k: hbm[k] for k in ("achieved", "peak", "unit", "frac")}, **common,
            "bytes_per_launch": bytes_per_launch, "alu": alu}


def oracle_problem(w):
    import oracle as O
    return O.Problem(nx=w.nx, ny=w.ny, dim=w.dim, flux=w.flux, ncomp=w.ncomp, bc=w.bc, x0=w.x0, x1=w.x1,
                     y0=w.y0, y1=w.y1, speed_x=w.speed_x, speed_y=w.speed_y, gamma=w.gamma, cfl=w.cfl,
                     eps_weno=w.eps_weno, eps_m=w.eps_m, recon=w.recon, switch_mode=w.switch_mode,
                     charwise=1 if w.variables == 1 else 0)


def oracle_initial(w, fp32: bool):
    return np.asarray(w.u0, np.float32 if fp32 else np.float64).astype(np.float64)


def oracle_worker(args):
    """Worker of the all-core CPU baseline (a child process that never touches the GPU): the first
    k RK steps of the workload by the FP64 oracle, timed around the oracle call only."""
    import oracle as O
    k = int(args.oracle_sample)
    w, _ = build_workload(args)
    pb = oracle_problem(w)
    u = oracle_initial(w, args.precision == "fp32")
    a = time.perf_counter()
    _, _, no = O.solve(pb, u, w.T, max_steps=k)
    el = time.perf_counter() - a
    print(json.dumps({"seconds": el, "steps": no, "cell_updates": w.ncell * 3.0 * no}), flush=True)


def oracle_all_cores(args, k):
    """k oracle steps in P concurrent child processes (one per host core, at most 16): the host's
    aggregate oracle throughput on this workload.  The oracle is single-threaded C; the processes
    run the same sample independently."""
    import subprocess
    P = args.cpu_workers or max(1, min(16, len(os.sched_getaffinity(0))))
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", args.workload, "--precision", args.precision,
           "--variables", args.variables, "--oracle-sample", str(k)]
    if args.n is not None:
        cmd += ["--n", str(args.n)]
    if args.recon is not None:
        cmd += ["--recon", args.recon]
    env = dict(os.environ, OMP_NUM_THREADS="1")
    procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True, env=env) for _ in range(P)]
    res = []
    for p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"oracle worker failed with status {p.returncode}")
        res.append(json.loads(out.strip().splitlines()[-1]))
    rate = sum(r["cell_updates"] / r["seconds"] for r in res)
    return {"value": rate, "cores": P, "worker_seconds": [float(f"{r['seconds']:.6g}") for r in res]}


def cpu_baseline(args, w, solver, u0_dev, prec):
    """The FP64 oracle on the host on a bounded sample of the same solve (its first k RK steps):
    once on one thread in this process, then in one process per host core.  Also the error of the
    GPU's state after the same k steps against the oracle's."""
    import oracle as O

    from paper_1602_00182_amd import binding as B
    pb = oracle_problem(w)
    u_ref = oracle_initial(w, prec == B.FP32)
    a = time.perf_counter()
    u1, t1, _ = O.step(pb, u_ref, w.T)
    per_step = time.perf_counter() - a
    k = max(2, int(args.cpu_seconds / max(per_step, 1e-6)))
    progress(f"oracle: first RK step on one thread took {per_step:.2f} s; sample = {k} steps")
    a = time.perf_counter()
    uo, _, no = O.solve(pb, u1, w.T, t=t1, max_steps=k - 1)
    el = time.perf_counter() - a + per_step
    ksteps = no + 1
    one = w.ncell * 3.0 * ksteps / el
    progress(f"oracle on one thread: {ksteps} steps in {el:.2f} s")
    allc = oracle_all_cores(args, ksteps)
    progress(f"oracle on {allc['cores']} processes done")
    base = {"value": allc["value"], "unit": "cell-updates/s", "cores": allc["cores"], "kind": "oracle",
            "sample": f"first {ksteps} RK3 steps of the same solve ({w.name}), FP64; {allc['cores']} oracle "
                      f"processes at once, one per host core, each running the whole sample",
            "single_thread": {"value": one, "cores": 1}, "worker_seconds": allc["worker_seconds"],
            "host": host_description()}
    solver.write(u0_dev, 0.0)
    solver.solve(w.T, ksteps)
    ug = solver.read().astype(np.float64)
    err = {"vs": "FP64 oracle", "rk_steps": ksteps, "l1": float(np.mean(np.abs(ug - uo))),
           "linf": float(np.max(np.abs(ug - uo)))}
    return base, err


def error_at_T(w, u_T, prec):
    """Float-bulk state at T against the double-bulk GPU path at T (which the parity tests hold
    bit-identical to the FP64 oracle): L1 and Linf over every cell and component."""
    import torch

    from paper_1602_00182_amd import binding as B
    if prec != B.FP32:
        return None
    u0 = torch.tensor(w.u0, dtype=torch.float64, device="cuda")
    with B.Solver(u0, **B.workload_params(w, B.FP64)) as s:
        st = s.solve(w.T)
        ref = s.read()
    progress(f"double-bulk reference solve to T done ({st['nsteps']} RK steps)")
    d = np.abs(np.asarray(u_T, np.float64) - ref)
    shape = (w.ny, w.nx) if w.dim == 2 else (w.nx,)
    smooth = np.tile(smooth_mask(ref, w.ncomp, shape), w.ncomp)
    out = {"vs": "double-bulk GPU path at T (bit-identical to the FP64 oracle in the parity tests)",
           "t": st["t"], "rk_steps": st["nsteps"], "l1": float(d.mean()), "linf": float(d.max()),
           "l1_rel": float(d.sum() / np.abs(ref).sum()),
           "values_differing_by_more_than": {t: float((d > float(t)).mean()) for t in ("1e-6", "1e-4", "1e-2", "1e-1")}}
    if smooth.any():
        ds = d[smooth]
        out["away_from_discontinuities"] = {
            "cells_fraction": float(smooth.mean()), "l1": float(ds.mean()), "linf": float(ds.max()),
            "rule": "cells more than 4 cells from any cell whose second undivided difference in some "
                    "component and direction exceeds 1e-3 max(1, |u|) in the double-bulk state"}
    return out


def smooth_mask(u, ncomp, shape, radius=4, tau=1e-3):
    """Cells away from discontinuities (flat boolean mask over the cells of `shape`): a cell is
    rough where some component's second undivided difference along some direction exceeds
    tau * max(1, |u|); every cell within `radius` cells of a rough one is excluded too."""
    U = np.asarray(u, dtype=np.float64).reshape((ncomp,) + tuple(shape))
    rough = np.zeros(tuple(shape), dtype=bool)
    for c in range(ncomp):
        f = U[c]
        for ax in range(len(shape)):
            p = np.concatenate([np.take(f, [0], axis=ax), f, np.take(f, [-1], axis=ax)], axis=ax)
            n = f.shape[ax]
            d2 = np.take(p, range(0, n), axis=ax) - 2.0 * f + np.take(p, range(2, n + 2), axis=ax)
            rough |= np.abs(d2) > tau * np.maximum(1.0, np.abs(f))
    for ax in range(len(shape)):
        acc = rough.copy()
        for k in range(1, radius + 1):
            acc |= np.roll(rough, k, axis=ax) | np.roll(rough, -k, axis=ax)
        rough = acc
    return ~rough.reshape(-1)


def cpu_baseline_batch(args, ws, bt, prec):
    """The FP64 oracle on the host over the first instances of the same batch, each solved to its
    T, instances spread over host threads (the oracle is plain C called through ctypes, which
    releases the GIL).  Also the error of the GPU's final states on those instances."""
    import concurrent.futures as cf

    import oracle as O

    from paper_1602_00182_amd import binding as B
    threads = max(1, min(16, len(os.sched_getaffinity(0))))

    def problem(w):
        return O.Problem(nx=w.nx, flux=w.flux, ncomp=w.ncomp, bc=w.bc, x0=w.x0, x1=w.x1, gamma=w.gamma, cfl=w.cfl,
                         eps_weno=w.eps_weno, eps_m=w.eps_m, recon=w.recon, switch_mode=w.switch_mode,
                         charwise=1 if w.variables == 1 else 0)

    def init(w):
        return np.asarray(w.u0, np.float32 if prec == B.FP32 else np.float64).astype(np.float64)

    # cost model from one timed instance: steps grow with N, so work grows with N^2
    a = time.perf_counter()
    first = O.solve(problem(ws[0]), init(ws[0]), ws[0].T)
    c = (time.perf_counter() - a) / float(ws[0].nx) ** 2
    budget = args.cpu_seconds * threads
    take, cost = 1, c * float(ws[0].nx) ** 2
    while take < len(ws) and cost + c * float(ws[take].nx) ** 2 <= budget:
        cost += c * float(ws[take].nx) ** 2
        take += 1
    sample = ws[1:take]
    a = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        rest = list(ex.map(lambda w: O.solve(problem(w), init(w), w.T), sample))
    el = time.perf_counter() - a
    results = [first] + rest
    work = sum(w.nx * 3.0 * r[2] for w, r in zip(ws[1:take], rest))
    base = {"value": work / el if sample else None, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"instances 1..{take - 1} of the seed-3 batch (of {len(ws)}), each solved to T by the FP64 "
                      f"oracle, {threads} instances at a time on host threads"}
    l1 = linf = 0.0
    cells = 0
    for b, (w, r) in enumerate(zip(ws[:take], results)):
        ug = bt.read(b).astype(np.float64)
        d = np.abs(ug - r[0])
        l1 += float(d.sum())
        linf = max(linf, float(d.max()))
        cells += d.size
    err = {"vs": "FP64 oracle", "instances": take, "final_time": "T = 0.2 of each", "l1": l1 / cells,
           "linf": linf}
    return base, err


def bench_batch(args, prec):
    import torch

    from paper_1602_00182_amd import binding as B
    from paper_1602_00182_amd import inputs as I
    ws = [apply_scheme(args, w) for w in I.euler_riemann_batch(count=4096 if args.n is None else args.n, seed=3)]
    dt = np.float32 if prec == B.FP32 else np.float64
    states = [np.asarray(w.u0, dt) for w in ws]
    stream = torch.cuda.Stream()
    bt = B.Batch(states, [B.workload_params(w, prec) for w in ws], stream=stream.cuda_stream)
    T = [w.T for w in ws]
    # reset = write the packed initial states back (host copy, outside the device work)
    packed = np.concatenate(states)
    packed_dev = torch.tensor(packed, device="cuda")

    def reset():
        B.lib().npweno_write(bt.h, B.ctypes.c_void_p(packed_dev.data_ptr()), 1, 0.0)

    for i in range(args.warmup):
        reset()
        bt.solve(T, args.max_rk_steps)
        progress(f"warmup batch solve {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    lat = []
    evs = []
    t0 = time.perf_counter()
    total_cell_stages = 0.0
    for i in range(args.steps):
        a = time.perf_counter()
        reset()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        stats, rc = bt.solve(T, args.max_rk_steps)
        e1.record(stream)
        evs.append((e0, e1))
        lat.append(time.perf_counter() - a)
        total_cell_stages += sum(w.nx * 3.0 * s["nsteps"] for w, s in zip(ws, stats))
        progress(f"timed batch solve {i + 1}/{args.steps}: {lat[-1]:.3f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = sum(e0.elapsed_time(e1) for e0, e1 in evs) / 1e3
    max_steps = max(s["nsteps"] for s in stats)
    esize = 4 if prec == B.FP32 else 8
    achieved = ACCESSES_PER_CELL_STAGE * esize * 3 * total_cell_stages / gpu_s / 1e9
    cb = err = None
    if not args.no_cpu_baseline and args.max_rk_steps < 0:
        cb, err = cpu_baseline_batch(args, ws, bt, prec)
    shape = bt.launch_shape()
    bt.close()
    label = kernel_label(ws[0], prec, shape, batched=True)
    tflops = alg_flops_per_cell_stage(ws[0]) * total_cell_stages / gpu_s / 1e12
    return {"value": total_cell_stages / wall, "ms_per_step": 1e3 * wall / args.steps,
            "cpu_baseline": cb, "error_vs_oracle": err, "scheme": scheme_of(ws[0]),
            "latency_s": _percentiles(lat), "instances": len(ws), "cells": int(sum(w.nx for w in ws)),
            "max_rk_steps": max_steps,
            "roofline": {"bound": "alu", "achieved": tflops, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tflops / ALU_PEAK_TFLOPS, "traffic": counter_traffic(label),
                         "traffic_note": "HBM bytes per launch while every instance is running (counters over "
                                         "the first 20 steps)",
                         "valu": valu_roof(label, cell_stages_per_s=total_cell_stages / gpu_s), "kernel": label,
                         "peak_basis": "FP32 vector FMA without packed-FP32 instructions",
                         "hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": achieved / HBM_PEAK_GBS},
                         "note": "work of all instances / GPU time of the timed region"}}


def bench_serving(args, prec):
    """The Poisson trace through the continuous-batching server, replayed in real time, then the
    first --serving-solo requests one solve at a time on the same GPU (and through the server alone,
    for a like-for-like comparison).  Every request's T is scaled by --serving-tscale so that the
    trace's work fits a benchmark run; arrivals, kinds and grid sizes are the trace's own."""
    from paper_1602_00182_amd import binding as B
    from paper_1602_00182_amd import inputs as I
    trace = I.serving_trace(nreq=args.serving_requests, seed=4, nmax=args.serving_nmax)
    for r in trace:
        r.work = r.work.with_(T=r.work.T * args.serving_tscale)
    dt = np.float32 if prec == B.FP32 else np.float64
    budget = int(args.serving_budget_mib) << 20

    def serve(reqs, label):
        srv = B.Server(budget, max_slots=512, precision=prec)
        pending = list(reqs)
        live, sid_of, lat, work, peak_running, peak_queued = {}, {}, {}, 0.0, 0, 0
        t0 = time.perf_counter()
        pumps = 0
        while pending or live:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                r = pending.pop(0)
                sid_of[r.rid] = live[r.rid] = srv.submit(np.asarray(r.work.u0, dt), r.work.T,
                                                         **B.workload_params(r.work, prec))
            if not live:  # idle until the next arrival
                time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
                continue
            nr, nq = srv.pump(args.pump_steps)
            pumps += 1
            peak_running, peak_queued = max(peak_running, nr), max(peak_queued, nq)
            for rid in [q for q, sid in live.items() if srv.finished(sid)]:
                del live[rid]
            if pumps % 200 == 0:
                progress(f"{label}: {len(reqs) - len(pending) - len(live)}/{len(reqs)} done, {nr} running, {nq} queued")
        wall = time.perf_counter() - t0
        by_rid = {r.rid: r for r in reqs}
        for rid, sid in sid_of.items():
            out, st, rc = srv.poll(sid)
            a, b, c = srv.times(sid)
            lat[rid] = (c - t0) - by_rid[rid].arrival
            work += by_rid[rid].work.nx * 3.0 * st["nsteps"]
        srv.close()
        progress(f"{label}: {len(reqs)} requests in {wall:.2f} s")
        return {"value": work / wall, "work_cell_updates": work, "wall_s": wall,
                "latency_s": _percentiles(list(lat.values())), "requests": len(reqs),
                "peak_running": peak_running, "peak_queued": peak_queued}

    full = serve(trace, "serving, full trace")
    K = min(args.serving_solo, len(trace))
    head = trace[:K]
    mix_k = serve(head, f"serving, first {K}")
    # one solve at a time, in arrival order (queueing included).  The autotuner's choice for every
    # size class is made first, outside the timed replay, as a long-running process would have it.
    for r in {(r.work.flux, r.work.ncomp, int(math.log2(r.work.nx))): r for r in head}.values():
        with B.Solver(np.asarray(r.work.u0, dt), **B.workload_params(r.work, prec)):
            pass
    t0 = time.perf_counter()
    lat1, work1 = [], 0.0
    for i, r in enumerate(head):
        now = time.perf_counter() - t0
        if now < r.arrival:
            time.sleep(r.arrival - now)
        with B.Solver(np.asarray(r.work.u0, dt), **B.workload_params(r.work, prec)) as s:
            st = s.solve(r.work.T)
        work1 += r.work.nx * 3.0 * st["nsteps"]
        lat1.append((time.perf_counter() - t0) - r.arrival)
        if (i + 1) % 50 == 0:
            progress(f"one at a time: {i + 1}/{K} done")
    wall1 = time.perf_counter() - t0
    span = max(r.arrival for r in trace) - min(r.arrival for r in trace)
    return {"value": full["value"], "requests": len(trace), "wall_s": full["wall_s"], "latency_s": full["latency_s"],
            "full_trace": full,
            "first_k": {"requests": K, "serving": mix_k,
                        "one_at_a_time": {"value": work1 / wall1, "wall_s": wall1, "latency_s": _percentiles(lat1)}},
            "offered_rate_req_s": 2000.0,
            "overload_factor": (full["work_cell_updates"] / span) / full["value"] if span > 0 else None,
            "hbm_budget_mib": args.serving_budget_mib, "pump_steps": args.pump_steps,
            "trace": f"{len(trace)} requests of the seed-4 Poisson trace at 2000 req/s, N log-uniform in [256, "
                     f"{args.serving_nmax}], each T scaled by {args.serving_tscale}"}


def build_workload(args):
    """The single-grid workload named on the command line and its description."""
    from paper_1602_00182_amd import inputs as I
    if args.workload == "advection":
        w = apply_scheme(args, I.advection_sine(n=args.n or 65536, T=0.5))
        desc = (f"1D linear advection N={w.nx} periodic, u0 = sin(pi x) (Table 5's problem at the headline's "
                f"size), {scheme_of(w)}, global LF, SSP-RK3 CFL 0.5 to T=0.5")
    elif args.workload == "advection2d":
        w = apply_scheme(args, I.advection2d_sine(n=args.n or 2048))
        desc = (f"2D linear advection v_t + v_x + v_y = 0 on {w.nx}^2 cells of [0,1]^2, periodic, "
                f"v0 = sin(2 pi (x + y)) (Section 6's problem), {scheme_of(w)}, CFL 0.4 to T=0.25")
    elif args.workload == "burgers":
        w = apply_scheme(args, I.burgers_noisy(n=args.n or 65536, seed=2))
        desc = (f"1D Burgers N={w.nx} periodic, u0 = 0.5 + sin(pi x) + seeded noise 1e-3, {scheme_of(w)}, "
                "global LF, SSP-RK3 CFL 0.5 to T=1.5/pi")
    else:
        w = apply_scheme(args, I.euler2d_quadrants(n=args.n or 2048))
        desc = (f"2D Euler {w.nx}^2 on [0,1]^2, four seeded constant quadrant states (rho, p in [0.1,1.5], "
                f"u, v in [-1,1]) split at (0.5,0.5), transmissive, gamma 1.4, {scheme_of(w)}, dimension by "
                "dimension with one midpoint point per face, global LF, SSP-RK3 CFL 0.4 to T=0.25")
    return w, desc


def main():
    args = parse()
    if args.oracle_sample is not None:
        oracle_worker(args)
        return
    if args.steps is None:
        args.steps = {"burgers": 20, "advection": 20, "euler_batch": 2, "euler2d": 3, "advection2d": 3}.get(
            args.workload, 1)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {max(args.gpus, world)} GPUs)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1602_00182_amd import binding as B
    from paper_1602_00182_amd import inputs as I
    torch.cuda.set_device(0)
    progress("torch and the library loaded")
    prec = B.FP32 if args.precision == "fp32" else B.FP64
    dname = "f32" if prec == B.FP32 else "f64"
    base = {"unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dname,
            "data": "synthetic (seeded)"}

    if args.workload in ("burgers", "advection", "euler2d", "advection2d"):
        w, desc = build_workload(args)
        res, solver, u0_dev = bench_single(args, w, prec)
        out = {"metric": METRIC, "value": res["value"], **base, "ms_per_step": res["ms_per_step"],
               "config": {"workload": w.name, "description": desc, "scheme": scheme_of(w), "cells": w.ncell,
                          "T": w.T, "cfl": w.cfl,
                          "rk_steps_per_solve": res["rk_steps_per_solve"], "eta_precision": "f64",
                          "launch_shape": res["launch_shape"]},
               "latency_s": res["latency_s"], "roofline": res["roofline"]}
        if args.max_rk_steps >= 0:
            out["note"] = "profiling run: solves stopped after --max-rk-steps; not a benchmark value"
        if not args.no_error_at_t and args.max_rk_steps < 0:
            out["error_at_T"] = error_at_T(w, res["u_T"], prec)
        if not args.no_cpu_baseline:
            cb, err = cpu_baseline(args, w, solver, u0_dev, prec)
            out["cpu_baseline"] = cb
            out["error_vs_oracle"] = err
        solver.close()
    elif args.workload == "euler_batch":
        res = bench_batch(args, prec)
        out = {"metric": METRIC,
               "value": res["value"], **base, "ms_per_step": res["ms_per_step"],
               "config": {"workload": "euler_riemann_batch_4096",
                          "description": "4096 1D Euler Riemann problems, N in [256,4096], CFL 0.5 to T=0.2",
                          "scheme": res["scheme"],
                          "instances": res["instances"],
                          "cells": res["cells"], "max_rk_steps": res["max_rk_steps"]},
               "latency_s": res["latency_s"], "roofline": res["roofline"]}
        if res["cpu_baseline"] is not None:
            out["cpu_baseline"] = res["cpu_baseline"]
            out["error_vs_oracle"] = res["error_vs_oracle"]
    else:
        res = bench_serving(args, prec)
        out = {"metric": METRIC,
               "value": res["value"], **base, "ms_per_step": None,
               "config": {"workload": "serving_trace", "requests": res["requests"], "trace": res["trace"],
                          "hbm_budget_mib": res["hbm_budget_mib"], "pump_steps": res["pump_steps"]},
               "latency_s": res["latency_s"], "wall_s": res["wall_s"], "full_trace": res["full_trace"],
               "first_k": res["first_k"], "overload_factor": res["overload_factor"]}

    if args.calibrate_copy:
        n = 64 << 20  # 64 Mi floats = 256 MiB read + 256 MiB written
        a = torch.empty(n, dtype=torch.float32, device="cuda").uniform_()
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 4 * n
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
