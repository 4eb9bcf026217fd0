import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


def load_golden(name):
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            rows.append((parts[0], int(parts[1]), float(parts[2]), float(parts[3]), float(parts[4])))
    return rows


def check_sums(stats, u, ncomp, area, rel=1e-12):
    """The device's per-component FP64 sums (stats["mass"]) against an independent correctly
    rounded sum (math.fsum) of the read-back state times the cell area.  The device adds in a
    fixed order (per thread, then per workgroup, then over workgroups), so the two differ by far
    less than rel of the sum of magnitudes; a wrong area factor or component mapping does not."""
    import math

    import numpy as np
    u = np.asarray(u, dtype=np.float64).reshape(ncomp, -1)
    for c in range(ncomp):
        want = math.fsum(u[c]) * area
        scale = math.fsum(np.abs(u[c])) * area
        got = stats["mass"][c]
        assert abs(got - want) <= rel * scale + 1e-300, (c, got, want)
    for c in range(ncomp, 4):
        assert stats["mass"][c] == 0.0, (c, stats["mass"][c])


def smooth_cells(u, ncomp, shape, radius=4, tau=1e-3):
    """Cells away from discontinuities, as a flat boolean mask over the cells of `shape` ((n,) in
    1D, (ny, nx) in 2D): a cell is rough where, in some component and direction, the second
    undivided difference |u_{i-1} - 2 u_i + u_{i+1}| exceeds tau * max(1, |u_i|) (a jump of
    size J gives about J/2 there; smooth data gives u'' dx^2).  Every cell within `radius` cells of
    a rough cell is excluded as well (the reconstruction reaches three cells)."""
    import numpy as np
    U = np.asarray(u, dtype=np.float64).reshape((ncomp,) + tuple(shape))
    rough = np.zeros(tuple(shape), dtype=bool)
    for c in range(ncomp):
        f = U[c]
        for ax in range(len(shape)):
            p = np.concatenate([np.take(f, [0], axis=ax), f, np.take(f, [-1], axis=ax)], axis=ax)
            n = f.shape[ax]
            d2 = (np.take(p, range(0, n), axis=ax) - 2.0 * f + np.take(p, range(2, n + 2), axis=ax))
            rough |= np.abs(d2) > tau * np.maximum(1.0, np.abs(f))
    grown = rough.copy()
    for ax in range(len(shape)):
        acc = grown.copy()
        for s in range(1, radius + 1):
            acc |= np.roll(grown, s, axis=ax) | np.roll(grown, -s, axis=ax)
        grown = acc
    return ~grown.reshape(-1)


def assert_fp32_close(got, ref, ncomp, mask=None, rel=1e-5):
    """Element-wise float-bulk bar: |got - ref| <= rel * max(1, |ref|) on every cell of `mask`
    (all cells if None), every component."""
    import numpy as np
    g = np.asarray(got, dtype=np.float64).reshape(ncomp, -1)
    r = np.asarray(ref, dtype=np.float64).reshape(ncomp, -1)
    m = np.ones(g.shape[1], dtype=bool) if mask is None else np.asarray(mask)
    err = np.abs(g - r)[:, m]
    bound = rel * np.maximum(1.0, np.abs(r[:, m]))
    worst = float(np.max(err / bound)) if err.size else 0.0
    assert worst <= 1.0, f"max |err| / bound = {worst:.3f} over {int(m.sum())} cells"
    return int(m.sum())
