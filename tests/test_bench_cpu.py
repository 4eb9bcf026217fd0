"""Host-side checks of bench.py: the one-GPU guard and the counter-summary lookup."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_traffic_requires_matching_kernel_and_source(tmp_path, monkeypatch):
    import bench
    h = bench.kernel_source_hash()
    assert len(h) == 16
    pdir = tmp_path / "profiles"
    pdir.mkdir()
    (pdir / "k_hbm_counters.txt").write_text(
        f"# header\ntraffic kernel=stage1d_kernel<float,Burgers,1,128> source={h} bytes_per_launch=1234\n"
        f"traffic kernel=other source=0000000000000000 bytes_per_launch=99\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    assert bench.counter_traffic("stage1d_kernel<float, Burgers, 1, 128>") == pytest.approx(1234.0)
    assert bench.counter_traffic("other") is None  # summary taken with other kernel sources
    assert bench.counter_traffic("stage1d_kernel<float, Burgers, 1, 256>") is None


def test_batch_cpu_baseline_threads_and_error(monkeypatch):
    """The batch baseline solves a prefix of the batch on host threads and measures the GPU's
    final states against the oracle's (here a stand-in batch that returns the oracle's own)."""
    import types

    import numpy as np

    import bench
    import oracle as O
    from paper_1602_00182_amd import inputs as I
    ws = I.euler_riemann_batch(count=6, seed=3)
    ws = [w.with_(T=0.02) for w in ws]

    class Exact:
        def read(self, b):
            w = ws[b]
            pb = O.Problem(nx=w.nx, flux=w.flux, ncomp=w.ncomp, bc=w.bc, x0=w.x0, x1=w.x1, gamma=w.gamma, cfl=w.cfl)
            return O.solve(pb, w.u0, w.T)[0]

    args = types.SimpleNamespace(cpu_seconds=60.0)
    base, err = bench.cpu_baseline_batch(args, ws, Exact(), 0)  # 0 = FP64 bulk
    assert base["kind"] == "oracle" and base["cores"] >= 1 and base["value"] > 0
    assert err["instances"] == len(ws)
    assert err["l1"] == 0.0 and err["linf"] == 0.0


def test_counter_valu_requires_matching_kernel_and_source(tmp_path, monkeypatch):
    import bench
    h = bench.kernel_source_hash()
    pdir = tmp_path / "profiles"
    pdir.mkdir()
    (pdir / "k_valu_counters.txt").write_text(
        f"# header\nvalu kernel=stage2d_kernel<float,Euler,4,64,8,recompute> source={h} wave_instr_per_launch=9.0e7 "
        f"wave_instr_per_cell_stage=21.5 classes=fma32:300.0,int32:100.0,rest:200.0\n"
        f"valu kernel=stage2d_kernel<float,Euler,4,62,8,recompute> source=0000000000000000 wave_instr_per_launch=1 "
        f"wave_instr_per_cell_stage=1 classes=fma32:1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    got = bench.counter_valu("stage2d_kernel<float, Euler, 4, 64, 8, recompute>")
    assert got["wave_instr_per_launch"] == 9.0e7 and got["wave_instr_per_cell_stage"] == 21.5
    assert got["classes"] == {"fma32": 300.0, "int32": 100.0, "rest": 200.0}
    # a summary of another kernel build does not count
    assert bench.counter_valu("stage2d_kernel<float, Euler, 4, 62, 8, recompute>") is None


def test_probe_argv_splits_the_remainder():
    """The counters leave compares, selects, moves and logic in one remainder; the probe gets it
    split in fixed proportions, and every other class as counted."""
    import bench
    argv = bench.probe_argv({"fma32": 300.0, "int32": 100.0, "rest": 210.0})
    mix = {a.split("=")[0]: float(a.split("=")[1]) for a in argv}
    tot = sum(bench.REST_SPLIT.values())
    assert mix["fma32"] == 300.0 and mix["int32"] == 100.0 and "rest" not in mix
    for k, w in bench.REST_SPLIT.items():
        assert mix[k] == pytest.approx(210.0 * w / tot, abs=1e-3)
    assert sum(mix.values()) == pytest.approx(610.0, abs=1e-2)


def test_oracle_worker_and_all_core_baseline():
    """The all-core CPU baseline runs the oracle sample in child processes (no GPU use): each
    reports its own time and work, and the aggregate is their summed rate."""
    import json
    import types

    import bench
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "burgers", "--n", "512",
                        "--oracle-sample", "3"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["steps"] == 3 and rec["cell_updates"] == 512 * 3 * 3 and rec["seconds"] > 0
    args = types.SimpleNamespace(cpu_workers=2, workload="burgers", precision="fp32", variables="componentwise",
                                 n=512, recon=None)
    res = bench.oracle_all_cores(args, 3)
    assert res["cores"] == 2 and len(res["worker_seconds"]) == 2
    assert res["value"] == pytest.approx(sum(512 * 9 / t for t in res["worker_seconds"]), rel=1e-2)


def test_roofline_bound_per_workload():
    """2D and Euler stages report the ALU roofline (with the HBM fraction beside it); 1D scalar
    stages report HBM.  Achieved = algorithmic work per launch / average launch time."""
    import bench
    from paper_1602_00182_amd import inputs as I
    w2 = I.euler2d_quadrants(n=64)
    r = bench.roofline(w2, "k", w2.ncell, 4, 1e-4, traffic=None)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert bench.alg_flops_per_cell_stage(w2) == 2 * (4 * 130 + 30)
    assert r["achieved"] == pytest.approx(1100 * 64 * 64 / 1e-4 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"]) and r["peak"] == pytest.approx(78.6432)
    assert r["hbm"]["achieved"] == pytest.approx(8 / 3 * 4 * 4 * 64 * 64 / 1e-4 / 1e9)
    w1 = I.burgers_noisy(n=4096)
    r1 = bench.roofline(w1, "k", w1.ncell, 4, 2e-6, traffic=5.0)
    assert r1["bound"] == "hbm" and r1["unit"] == "GB/s" and r1["traffic"] == 5.0
    assert r1["achieved"] == pytest.approx(8 / 3 * 4 * 4096 / 2e-6 / 1e9)


def test_smooth_mask_excludes_the_neighbourhood_of_jumps():
    import bench
    n = 40
    u = np.where(np.arange(n) < 20, 1.0, 0.2) + 1e-4 * np.sin(np.arange(n) / 7.0)
    m = bench.smooth_mask(u, 1, (n,))
    # the jump between cells 19 and 20 marks both as rough; 4 cells either side go too
    assert not m[15:25].any() and m[:15].all() and m[25:].all()
    two = np.stack([u, np.ones(n)])
    assert np.array_equal(bench.smooth_mask(two.reshape(-1), 2, (n,)), m)


def test_kernel_label_names_the_strip_and_tile_kernels():
    import types

    import bench
    w = types.SimpleNamespace(dim=2, flux=2, ncomp=4, recon=0, variables=0)
    strip = {"block": 256, "tile_x": 62, "tile_y": 16, "lds_shared": 0}
    tile = {"block": 256, "tile_x": 62, "tile_y": 8, "lds_shared": 0}
    assert bench.kernel_label(w, 1, strip) == "stage2d_strip_kernel<float, Euler, 4, 62, 16>"
    assert bench.kernel_label(w, 1, tile) == "stage2d_kernel<float, Euler, 4, 62, 8, recompute>"
