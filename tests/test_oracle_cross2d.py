"""Pins of the oracle's Section 6 reconstruction (k = 2, shape parameter from the five-cell cross,
eq. i+1/2_eps_approx_2d), against what the paper and the mathematics fix:

* the paper's claim for its reconstruction-error figure: on cell averages of sin(2 pi (x + y)) the
  perturbed edge values converge at third order, the unperturbed ENO2 values at second order;
* the printed estimate -(-2 u_{i-1} + u_i - 5 u_{i+1})/6 of the edge value has zero first moment
  about the edge, i.e. it is exact on linear data (what makes the printed formula consistent);
* x/y transposition symmetry, constancy and conservation;
* Table 8's ranking (the perturbed method is the more accurate in the advection run).
Table 8's numbers themselves are not reproduced (see the design notes): parity of the GPU path is
pinned against this oracle and these properties.
"""
import math

import numpy as np
import pytest

import oracle as O


def _avg(n):
    h = 1.0 / n
    xc = (np.arange(n) + 0.5) * h
    s = (math.sin(math.pi * h) / (math.pi * h)) ** 2
    X, Y = np.meshgrid(xc, xc)
    return np.sin(2 * math.pi * (X + Y)) * s


def _problem(n, **kw):
    base = dict(nx=n, ny=n, dim=2, flux=O.ADVECTION, speed_x=1.0, speed_y=1.0, x0=0.0, x1=1.0, y0=0.0,
                y1=1.0, bc=O.PERIODIC, recon=O.RBF_ENO2_2D, switch_mode=O.SWITCH_OFF)
    base.update(kw)
    return O.Problem(**base)


def _edge_errors(n, direction):
    h = 1.0 / n
    vm, vp = O.face_states(_problem(n), direction, _avg(n))
    faces = np.arange(n + 1) * h
    centres = (np.arange(n) + 0.5) * h
    exact = np.sin(2 * math.pi * (faces[None, :] + centres[:, None]))
    return math.sqrt(np.mean((vm - exact) ** 2)), math.sqrt(np.mean((vp - exact) ** 2))


@pytest.mark.parametrize("direction", [0, 1])
def test_reconstruction_is_third_order(direction):
    errs = [_edge_errors(n, direction) for n in (16, 32, 64, 128)]
    for side in (0, 1):
        orders = [math.log2(errs[k][side] / errs[k + 1][side]) for k in range(3)]
        assert min(orders[1:]) > 2.8, orders


def test_eno2_edges_are_second_order():
    """The same stencils without the perturbation (1D ENO2 along x at the edge midpoint)."""
    errs = []
    for n in (32, 64, 128):
        h = 1.0 / n
        f = _avg(n)
        pb = O.Problem(nx=n, flux=O.ADVECTION, recon=O.ENO2, x0=0.0, x1=1.0, switch_mode=O.SWITCH_OFF)
        vm = np.array([O.line_states(pb, f[j])[0] for j in range(n)])
        faces = np.arange(n + 1) * h
        centres = (np.arange(n) + 0.5) * h
        exact = np.sin(2 * math.pi * (faces[None, :] + centres[:, None]))
        errs.append(math.sqrt(np.mean((vm - exact) ** 2)))
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert all(1.8 < o < 2.3 for o in orders), orders


def test_printed_edge_estimate_is_exact_on_linear_data():
    # -(-2 a + b - 5 c)/6 on a, b, c = l(x_{i-1}), l(x_i), l(x_{i+1}) equals l(x_{i+1/2}) for linear l
    for a0, a1 in [(0.3, 1.7), (-2.0, 0.25), (5.0, -3.0)]:
        h = 0.1
        xs = np.array([-1.5, -0.5, 0.5]) * h  # cell centres relative to the edge x_{i+1/2}
        a, b, c = a0 + a1 * xs
        assert -(-2 * a + b - 5 * c) / 6 == pytest.approx(a0, abs=1e-14)
    # and the edge routine reproduces linear data exactly in both directions (second
    # differences vanish, so the perturbation is zero)
    w3 = np.array([1.0, 1.5, 2.0])
    assert O.cross_edge(w3, [1.5, 1.5], True) == pytest.approx(1.75, abs=1e-15)
    assert O.cross_edge(w3, [1.5, 1.5], False) == pytest.approx(1.25, abs=1e-15)


@pytest.mark.parametrize("x0,centred", [(0.3, True), (-0.6, False)])
def test_perturbation_cancels_the_taylor_error_of_both_stencils(x0, centred):
    """v = sin(x) + cos(2y) as exact cell averages: where the slope flattens ENO picks the centred
    pair {k, k+1}, where it steepens the extrapolating pair {k-1, k}; the right-edge value converges
    at third order for both (K = 4 and K = -8 cancel their different Taylor errors)."""
    errs = []
    for h in (0.04, 0.02, 0.01):
        y0 = 0.2
        ax = lambda c: (-np.cos(c + h / 2) + np.cos(c - h / 2)) / h  # noqa: E731
        ay = lambda c: (np.sin(2 * (c + h / 2)) - np.sin(2 * (c - h / 2))) / (2 * h)  # noqa: E731
        cells = np.array([ax(x0 + k * h) + ay(y0) for k in (-1, 0, 1)])
        trans = np.array([ax(x0) + ay(y0 - h), ax(x0) + ay(y0 + h)])
        picks_centred = abs(cells[2] - cells[1]) <= abs(cells[1] - cells[0])
        assert picks_centred == centred
        v = O.cross_edge(cells, trans, True, use_switch=False)
        errs.append(abs(v - (math.sin(x0 + h / 2) + math.cos(2 * y0))))
    assert math.log2(errs[0] / errs[1]) > 2.6 and math.log2(errs[1] / errs[2]) > 2.6, errs


def test_transpose_symmetry_constancy_conservation():
    n = 24
    rng = np.random.default_rng(3)
    f = 1.5 + 0.3 * rng.random((n, n))
    pb = _problem(n, switch_mode=O.SWITCH_MONOTONE)
    vmx, vpx = O.face_states(pb, 0, f)
    vmy, vpy = O.face_states(pb, 1, f.T)
    assert np.array_equal(vmx, vmy) and np.array_equal(vpx, vpy)
    L, _ = O.rhs(pb, np.full(n * n, 0.7))
    assert np.max(np.abs(L)) <= 1e-12
    u, _, _ = O.solve(pb, f.reshape(-1), 0.1)
    assert abs(u.sum() - f.sum()) <= 1e-13 * abs(f.sum())


def test_needs_two_dimensions():
    with pytest.raises(O.OracleError):
        O.rhs(O.Problem(nx=16, flux=O.ADVECTION, recon=O.RBF_ENO2_2D), np.zeros(16))


def test_table8_ranking_more_accurate_than_eno():
    """Advection v_t + v_x + v_y = 0 on [0,1]^2 (Section 7, Example 1), dt = 0.1 h, T = 0.5, the
    switch on: the perturbed reconstruction beats ENO2 at N = 20, 40, 80."""
    for n in (20, 40, 80):
        h = 1.0 / n
        u0 = _avg(n).reshape(-1)
        out = {}
        for recon in (O.ENO2, O.RBF_ENO2_2D):
            pb = _problem(n, recon=recon, switch_mode=O.SWITCH_MONOTONE, dt_fixed=0.1 * h)
            u, _, _ = O.solve(pb, u0, 0.5)
            out[recon] = float(np.mean(np.abs(u - u0)))  # the exact solution returns to u0 at T = 0.5
        assert out[O.RBF_ENO2_2D] < out[O.ENO2], (n, out)


def test_example1_error_is_the_midpoint_quadrature_phase_lag():
    """Section 7, Example 1 (v_t + v_x + v_y = 0 on [0,1]^2, sin(2 pi (x + y)), dt = 0.1 h, T = 0.5,
    one flux point at each edge midpoint).  The reconstruction targets the point value at the edge
    midpoint (eq. i+1/2_eps_2d cancels both Taylor terms), so the only second-order error left is
    the midpoint rule's: the flux integral over an edge exceeds h times its midpoint value by
    h^3/24 times the transverse second derivative.  For the mode exp(i k (x + y)) this adds
    k^3 h^2 / 12 to the phase speed, a lag phi = k^3 h^2 T / 12, and an L1 error of
    (2/pi) 2 sin(phi/2) times the amplitude.  What is left after that lag is the reconstruction's
    own error, third order.  (A reconstruction of the edge average instead, without the transverse
    term, would have no lag and an error five times smaller at N = 80.)"""
    res = {}
    for n in (40, 80):
        h, T = 1.0 / n, 0.5
        s = (math.sin(math.pi * h) / (math.pi * h)) ** 2
        xc = (np.arange(n) + 0.5) * h
        X, Y = np.meshgrid(xc, xc)
        pb = _problem(n, switch_mode=O.SWITCH_OFF, dt_fixed=0.1 * h)
        u, _, _ = O.solve(pb, _avg(n).reshape(-1), T)
        phi = (2 * math.pi) ** 3 * h * h * T / 12
        exact = (s * np.sin(2 * math.pi * (X + Y - 2 * T))).reshape(-1)
        lagged = (s * np.sin(2 * math.pi * (X + Y - 2 * T) - phi)).reshape(-1)
        res[n] = (float(np.mean(np.abs(u - exact))), 2 / math.pi * 2 * math.sin(phi / 2) * s,
                  float(np.mean(np.abs(u - lagged))))
    l1, closed, _ = res[80]
    assert abs(l1 - closed) <= 0.03 * closed, res
    assert math.log2(res[40][2] / res[80][2]) > 2.8, res


def test_mirror_symmetry_of_the_two_edges():
    """Reflecting the data in x swaps the roles of the edges: v^- of the original at interface f
    is v^+ of the reflection at interface n - f (the left-edge formulas mirror the right-edge ones)."""
    n = 20
    rng = np.random.default_rng(11)
    f = 1.0 + np.sin(2 * math.pi * (np.arange(n)[None, :] + 0.3 * np.arange(n)[:, None]) / n) \
        + 0.05 * rng.random((n, n))
    for sw in (O.SWITCH_OFF, O.SWITCH_MONOTONE):
        pb = _problem(n, switch_mode=sw)
        vm, vp = O.face_states(pb, 0, f)
        rvm, rvp = O.face_states(pb, 0, f[:, ::-1].copy())
        # equal up to the rounding of differently ordered sums (a - 2b + c vs c - 2b + a)
        assert np.max(np.abs(vm - rvp[:, ::-1])) <= 1e-13
        assert np.max(np.abs(vp - rvm[:, ::-1])) <= 1e-13
