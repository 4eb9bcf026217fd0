"""GPU parity of the column-strip form of the 2D Euler stage (launch shapes 6, 7, 8: strips of 62
columns and 16, 32 or 64 rows, walked in 4-row chunks) against the FP64 oracle: the same scheme
as the tile kernels (Section 7, eq. 2DIntegral, one midpoint point per face), so the double bulk
must give the oracle's bits on every grid, including strips cut short by the grid's top edge,
grids narrower than a strip and periodic grids shorter than the ghost depth."""
import sys

import numpy as np
import pytest

import oracle as O
from conftest import assert_fp32_close, smooth_cells
from paper_1602_00182_amd import binding as B
from paper_1602_00182_amd import inputs as I

pytestmark = pytest.mark.gpu

_H = {6: 16, 7: 32, 8: 64}


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _oracle_problem(w):
    return O.Problem(nx=w.nx, flux=w.flux, dim=w.dim, ny=w.ny, ncomp=w.ncomp, bc=w.bc, x0=w.x0, x1=w.x1,
                     y0=w.y0, y1=w.y1, speed_x=w.speed_x, speed_y=w.speed_y, gamma=w.gamma, cfl=w.cfl,
                     eps_weno=w.eps_weno, eps_m=w.eps_m, recon=w.recon, switch_mode=w.switch_mode,
                     dt_fixed=w.dt_fixed)


def _quadrants(n, ny, bc=I.TRANSMISSIVE, seed=5):
    m = max(n, ny, 4)
    w = I.euler2d_quadrants(n=m, seed=seed)
    U = w.u0.reshape(4, m, m)[:, :ny, :n].copy().reshape(-1)
    return w.with_(nx=n, ny=ny, u0=U, bc=bc)


def _check_fp64(w, steps):
    with B.Solver(w.u0, **B.workload_params(w)) as s:
        ls = s.launch_shape()
        L = s.rhs()
        st = s.solve(w.T, max_steps=steps)
        u = s.read()
    Lo, _ = O.rhs(_oracle_problem(w), w.u0)
    assert np.array_equal(L, Lo)
    uo, to, no = O.solve(_oracle_problem(w), w.u0, w.T, max_steps=steps)
    assert st["nsteps"] == no and st["t"] == to
    assert np.array_equal(u, uo)
    ao = O.alpha(_oracle_problem(w), uo)
    assert st["alpha"][0] == ao[0] and st["alpha"][1] == ao[1]
    return ls


@pytest.mark.parametrize("shape", [6, 7, 8])
@pytest.mark.parametrize("recon", [I.RBF_WENO5, I.WENO5_JS, I.RBF_ENO3, I.ENO3])
def test_strip_shapes_fp64(shape, recon, monkeypatch):
    """Every strip height and every k = 3 scheme on a 131 x 150 grid: several strips per column
    of tiles, the last one cut short by the grid's top, and three columns of strips (the last 7
    wide)."""
    _say(f"strip shape={shape} recon={recon}")
    monkeypatch.setenv("NPW_TILE2D", str(shape))
    ls = _check_fp64(_quadrants(131, 150).with_(recon=recon), 3)
    assert (ls["tile_x"], ls["tile_y"], ls["lds_shared"]) == (62, _H[shape], 0)


@pytest.mark.parametrize("shape", [6, 8])
def test_strip_rbf_weno5_without_the_switch_fp64(shape, monkeypatch):
    """RBF-WENO5 with the switch on runs a strip kernel built for that scheme alone; with the
    switch off it runs the strip that reads the scheme from the record.  Both bit for bit."""
    _say(f"strip rbf_weno5 switch off shape={shape}")
    monkeypatch.setenv("NPW_TILE2D", str(shape))
    nx, ny = 131, 150  # smooth periodic data: without the switch the quadrants' jumps oscillate
    x = I.cell_centers(nx, 0.0, 1.0)[None, :]
    y = I.cell_centers(ny, 0.0, 1.0)[:, None]
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
    U = I.euler_prim_to_cons(rho, 0.4 + 0 * rho, 1.0 + 0.2 * np.cos(2 * np.pi * x) + 0 * rho, v=-0.3 + 0 * rho)
    w = _quadrants(nx, ny, I.PERIODIC).with_(u0=U.reshape(-1), switch_mode=I.SWITCH_OFF)
    _check_fp64(w, 3)


@pytest.mark.parametrize("n,ny,bc", [(5, 3, I.PERIODIC), (62, 32, I.TRANSMISSIVE), (63, 33, I.PERIODIC),
                                     (124, 65, I.TRANSMISSIVE), (1, 7, I.PERIODIC), (9, 1, I.TRANSMISSIVE),
                                     (1, 1, I.PERIODIC), (2, 2, I.TRANSMISSIVE), (70, 4, I.PERIODIC),
                                     (64, 37, I.PERIODIC)])
def test_strip_grid_edges_fp64(n, ny, bc, monkeypatch):
    """32-row strips on grids smaller than one strip (periodic rows and columns wrapping through
    the ghosts several times), on exactly one strip, one cell past a strip in each direction, two
    by two strips plus one row, one chunk tall, and degenerate grids one cell wide or tall."""
    _say(f"strip grid {n}x{ny} bc={bc}")
    monkeypatch.setenv("NPW_TILE2D", "7")
    _check_fp64(_quadrants(n, ny, bc), 4)


def test_strip_periodic_many_strips_fp64(monkeypatch):
    """16-row strips on a periodic 200 x 130 grid (four columns of strips, nine strips high, the
    last two rows tall): the strips' ghost rows wrap around the grid's top and bottom."""
    _say("strip periodic 200x130")
    monkeypatch.setenv("NPW_TILE2D", "6")
    _check_fp64(_quadrants(200, 130, I.PERIODIC), 3)


@pytest.mark.parametrize("recon,variables", [(I.RBF_WENO3, I.COMPONENTWISE), (I.RBF_WENO5, I.CHARACTERISTIC)])
def test_strip_shapes_fall_back_for_other_schemes(recon, variables, monkeypatch):
    """The strips run component-wise k = 3 only; a k = 2 or characteristic-wise solve asked for a
    strip shape runs the 62 x 8 tile and reports it."""
    _say(f"strip fallback recon={recon} variables={variables}")
    monkeypatch.setenv("NPW_TILE2D", "7")
    w = _quadrants(131, 37).with_(recon=recon, variables=variables)
    with B.Solver(w.u0, **B.workload_params(w)) as s:
        ls = s.launch_shape()
        assert (ls["tile_x"], ls["tile_y"]) == (62, 8)
        s.solve(w.T, max_steps=2)
        u = s.read()
    pb = _oracle_problem(w)
    pb.charwise = 1 if variables == I.CHARACTERISTIC else 0
    uo, _, _ = O.solve(pb, w.u0, w.T, max_steps=2)
    assert np.array_equal(u, uo)


@pytest.mark.parametrize("shape", [6, 7, 8])
def test_strip_fp32_against_tiles_and_oracle(shape, monkeypatch):
    """Float bulk, 131 x 150, 5 steps: the strip kernel against the 62 x 8 tile kernel (the same
    functions; fused multiply-adds may be formed differently, so a unit in the last place apart,
    and an ENO stencil may flip where they differ) and element-wise against the FP64 oracle away
    from the quadrant discontinuities."""
    _say(f"strip fp32 shape={shape}")
    w = _quadrants(131, 150)
    u32 = np.asarray(w.u0, np.float32)
    out = {}
    for sh in ("4", str(shape)):
        monkeypatch.setenv("NPW_TILE2D", sh)
        with B.Solver(u32, **B.workload_params(w, B.FP32)) as s:
            s.solve(w.T, max_steps=5)
            out[sh] = s.read().astype(np.float64)
    scale = max(1.0, float(np.max(np.abs(out["4"]))))
    assert np.mean(np.abs(out[str(shape)] - out["4"])) <= 1e-6 * scale
    uo, _, _ = O.solve(_oracle_problem(w), u32.astype(np.float64), w.T, max_steps=5)
    mask = smooth_cells(uo, 4, (w.ny, w.nx))
    assert mask.mean() > 0.5
    assert_fp32_close(out[str(shape)], uo, 4, mask)
