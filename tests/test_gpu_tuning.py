"""The block-size autotuner: its choice is cached, and every block size gives the same bits."""
import os
import sys

import numpy as np
import pytest

from paper_1602_00182_amd import binding as B
from paper_1602_00182_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_autotuner_caches_and_block_size_never_changes_results(tmp_path, monkeypatch):
    print("[case] autotuner", flush=True)
    sys.stdout.flush()
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("NPW_TUNE_CACHE", str(cache))
    monkeypatch.delenv("NPW_BLOCK", raising=False)
    monkeypatch.delenv("NPW_AUTOTUNE", raising=False)
    w = I.burgers_noisy(n=20000, seed=3)
    u32 = np.asarray(w.u0, np.float32)
    with B.Solver(u32, **B.workload_params(w, B.FP32)) as s:
        s.solve(w.T, max_steps=40)
        tuned = s.read()
    lines = cache.read_text().split()
    assert len(lines) == 2 and int(lines[1]) in (64, 128, 256, 512)
    for bs in ("64", "128", "256", "512"):
        monkeypatch.setenv("NPW_BLOCK", bs)
        with B.Solver(u32, **B.workload_params(w, B.FP32)) as s:
            s.solve(w.T, max_steps=40)
            assert np.array_equal(s.read(), tuned), bs
    # batches are tuned too, and agree with the single solves
    monkeypatch.delenv("NPW_BLOCK")
    ws = [I.burgers_noisy(n=700 + 300 * b, seed=b) for b in range(4)]
    with B.Batch([np.asarray(x.u0, np.float32) for x in ws], [B.workload_params(x, B.FP32) for x in ws]) as bt:
        bt.solve(0.05)
        for b, x in enumerate(ws):
            with B.Solver(np.asarray(x.u0, np.float32), **B.workload_params(x, B.FP32)) as s:
                s.solve(0.05)
                assert np.array_equal(bt.read(b), s.read())
    assert any(k.endswith("_i1") for k in cache.read_text().split()[::2])  # the batch got its own entry
