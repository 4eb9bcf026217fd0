"""Pins of the oracle's building blocks against independent derivations (CPU only).

* Table 3 against brute-force multiquadric-RBF interpolation of the primitive function in
  200-digit arithmetic (Sections 2 and 3.2, Table 3).
* The eta formula of Table 3 against its closed form on sinusoidal data, and the combined
  (row, eta) reconstruction against the fourth-order Taylor claim of Section 3.5.
* The monotone switch (Section 4, eqs. root_value / adaptation) against the extremum of the
  exact quadratic reconstruction, found with rational arithmetic.
* The Jiang-Shu smoothness indicators against their integral definition.
"""
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

import oracle as O


# ---------------------------------------------------------------------------------------
# Table 3 from brute-force MQ-RBF interpolation
# ---------------------------------------------------------------------------------------
def _mq_coefficients(r, eta, dps=200):
    """Coefficients of ubar_{i-r+j} (j = 0..2) in P'(x_{i+1/2}) where P is the multiquadric
    interpolant sqrt(1 + eps^2 (x - x_l)^2) of the primitive V at the four cell boundaries of
    the stencil {i-r, .., i-r+2}; unit cell width, x_{i+1/2} = 0, eps^2 = eta."""
    mp.mp.dps = dps
    e2 = mp.mpf(eta)
    nodes = [mp.mpf(-r - 1 + l) for l in range(4)]
    A = mp.matrix(4, 4)
    for k in range(4):
        for l in range(4):
            A[k, l] = mp.sqrt(1 + e2 * (nodes[k] - nodes[l]) ** 2)
    # V(node_l) = sum_{j < l} ubar_{i-r+j} (unit cell width)
    B = mp.matrix(4, 3)
    for l in range(4):
        for j in range(3):
            B[l, j] = 1 if j < l else 0
    g = mp.matrix(1, 4)
    for l in range(4):
        d = 0 - nodes[l]
        g[0, l] = e2 * d / mp.sqrt(1 + e2 * d * d)
    out = []
    for j in range(3):
        col = mp.lu_solve(A, mp.matrix([B[l, j] for l in range(4)]))
        out.append(sum(g[0, l] * col[l] for l in range(4)))
    return out


@pytest.mark.parametrize("r", [-1, 0, 1, 2])
def test_table3_matches_multiquadric_flat_limit(r):
    e1, e2 = mp.mpf("1e-40"), mp.mpf("2e-40")
    c1 = _mq_coefficients(r, e1)
    c2 = _mq_coefficients(r, e2)
    poly = [float(2 * c1[j] - c2[j]) for j in range(3)]
    pert = [float((c2[j] - c1[j]) / (e2 - e1)) for j in range(3)]
    got_c = [O.row_value(r, *(1.0 if k == j else 0.0 for k in range(3)), 0.0) for j in range(3)]
    got_p = [O.row_value(r, *(1.0 if k == j else 0.0 for k in range(3)), 1.0) - got_c[j] for j in range(3)]
    np.testing.assert_allclose(got_c, poly, rtol=0, atol=1e-13)
    np.testing.assert_allclose(got_p, pert, rtol=0, atol=1e-12)


def test_table3_rows_consistent():
    """Polynomial rows sum to one (consistency), perturbation rows to zero: the k = 3 MQ
    perturbation leaves constants untouched.  The brute-force limit above fixes the printed
    r = -1 entry at 11/6."""
    c, p = O.table3()
    np.testing.assert_allclose(c.sum(axis=1), 1.0, atol=1e-15)
    np.testing.assert_allclose(p.sum(axis=1), 0.0, atol=1e-15)
    assert c[0, 0] == pytest.approx(11.0 / 6.0)


# ---------------------------------------------------------------------------------------
# eta closed forms
# ---------------------------------------------------------------------------------------
def _sin_avgs(kappa, h, centers, phase=0.0):
    s = kappa * h / 2
    return np.sin(kappa * centers + phase) * math.sin(s) / s


@pytest.mark.parametrize("n,kappa", [(80, math.pi), (40, 2 * math.pi), (256, 3 * math.pi)])
def test_eta_closed_form_on_sinusoids(n, kappa):
    """For exact cell averages of sin(kappa x) both undivided differences are proportional to
    cos(kappa x_{i+1/2}): D3 = 8 s^3 A cos, D1 = (24 s + 8 s^3) A cos with s = sin(kappa h / 2),
    so eta = s^2 / (3 + s^2) wherever the cosine is not small."""
    h = 2.0 / n
    xc = -1.0 + (np.arange(n) + 0.5) * h
    u = _sin_avgs(kappa, h, xc, 0.37)
    s = math.sin(kappa * h / 2)
    expect = s * s / (3 + s * s)
    checked = 0
    for i in range(1, n - 2):
        xi = xc[i] + h / 2
        if abs(math.cos(kappa * xi + 0.37)) < 0.2:
            continue
        got = O.eta(u[i - 1], u[i], u[i + 1], u[i + 2], 1e-12)
        assert got == pytest.approx(expect, rel=2e-6)
        checked += 1
    assert checked > n // 3
    if n == 80 and kappa == math.pi:
        assert expect == pytest.approx(5.135138791e-4, rel=1e-9)


def test_eta_vanishes_on_quadratic_data():
    """Cell averages of a quadratic are a quadratic sequence: the third undivided difference is
    exactly zero, so eta = 0 and the scheme is the polynomial WENO5 there."""
    for a, b, c in [(1, 0, 0), (3, -2, 5), (-0.5, 0.25, 7.0)]:
        u = [a * k * k + b * k + c for k in range(-1, 3)]
        assert O.eta(*u, 1e-12) == 0.0


def test_eta_constant_state_is_zero():
    assert O.eta(0.7, 0.7, 0.7, 0.7, 1e-12) == 0.0


def test_eta_eps_m_sign_follows_denominator():
    # denominator exactly zero -> +eps_M; negative denominator -> -eps_M (never crosses zero)
    assert O.eta(0.0, 1.0, 1.0, 0.0 + 0.0, 1e-12) == pytest.approx(
        (0 - 3 + 3 - 0) / ((0 - 15 + 15 - 0) + 1e-12))
    d = O.eta(0.0, 0.0, 0.0, 1e-13, 1e-12)  # den = -1e-13 -> -1.1e-12
    assert d == pytest.approx(-1e-13 / (-1e-13 - 1e-12))


# ---------------------------------------------------------------------------------------
# Fourth-order claim of Section 3.5 for every row with the shared interface eta
# ---------------------------------------------------------------------------------------
def _avg_test_fn(a, b):
    # v(x) = sin(x + 0.3) + 0.5 cos(2 x): exact average over [a, b]
    return (-math.cos(b + 0.3) + math.cos(a + 0.3) + 0.25 * (math.sin(2 * b) - math.sin(2 * a))) / (b - a)


def _v(x):
    return math.sin(x + 0.3) + 0.5 * math.cos(2 * x)


@pytest.mark.parametrize("r", [-1, 0, 1, 2])
def test_rows_with_eta_are_fourth_order(r):
    X = 0.4  # interface x_{i+1/2}
    errs_eta, errs_poly = [], []
    hs = [0.08, 0.04, 0.02, 0.01]
    for h in hs:
        avg = {m: _avg_test_fn(X + (m - 1) * h, X + m * h) for m in range(-3, 5)}  # cell i+m
        eta = O.eta(avg[-1], avg[0], avg[1], avg[2], 1e-12)
        w = [avg[-r + j] for j in range(3)]
        errs_eta.append(abs(O.row_value(r, *w, eta) - _v(X)))
        errs_poly.append(abs(O.row_value(r, *w, 0.0) - _v(X)))
    orders_eta = [math.log2(errs_eta[k] / errs_eta[k + 1]) for k in range(3)]
    orders_poly = [math.log2(errs_poly[k] / errs_poly[k + 1]) for k in range(3)]
    assert min(orders_eta[1:]) > 3.7, orders_eta
    assert max(abs(o - 3.0) for o in orders_poly[1:]) < 0.2, orders_poly


# ---------------------------------------------------------------------------------------
# Monotone switch against the exact quadratic reconstruction
# ---------------------------------------------------------------------------------------
def _quadratic_extremum(a, b, c):
    """Quadratic p with cell averages a, b, c on [0,1], [1,2], [2,3] (exact rationals);
    returns its critical point or None when p is linear."""
    a, b, c = Fraction(a), Fraction(b), Fraction(c)
    # p(x) = k0 + k1 x + k2 x^2; integral over [m, m+1] = k0 + k1 (2m+1)/2 + k2 (3m^2+3m+1)/3
    M = [[Fraction(1), Fraction(2 * m + 1, 2), Fraction(3 * m * m + 3 * m + 1, 3)] for m in range(3)]
    rhs = [a, b, c]
    # Gaussian elimination in rationals
    for col in range(3):
        piv = next(r for r in range(col, 3) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        rhs[col], rhs[piv] = rhs[piv], rhs[col]
        for r in range(3):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [M[r][k] - f * M[col][k] for k in range(3)]
                rhs[r] = rhs[r] - f * rhs[col]
    k1 = rhs[1] / M[1][1]
    k2 = rhs[2] / M[2][2]
    if k2 == 0:
        return None
    return -k1 / (2 * k2)


def test_monotone_flag_matches_quadratic_extremum():
    rng = np.random.default_rng(11)
    mismatches = 0
    n_flag = 0
    for _ in range(3000):
        a, b, c = (int(v) for v in rng.integers(-20, 21, size=3))
        xs = _quadratic_extremum(a, b, c)
        # Exact ties (extremum on the window's outer edge) fail the strict inequalities of eq.
        # (adaptation) and count as monotone; they are kept in the draw.
        expect = int(xs is not None and 0 < xs < 3)
        n_flag += expect
        if O.monotone_flag(float(a), float(b), float(c)) != expect:
            mismatches += 1
    assert mismatches == 0
    assert 300 < n_flag < 2950  # both outcomes well represented


def _tie_windows():
    """Integer windows whose quadratic has its extremum exactly at x_p = 0 or x_p = 3 dx, the
    outer edges x_{j-3/2}, x_{j+3/2} of the stencil (found with rational arithmetic)."""
    out = []
    for a in range(-6, 7):
        for b in range(-6, 7):
            for c in range(-6, 7):
                xs = _quadratic_extremum(a, b, c)
                if xs is not None and (xs == 0 or xs == 3):
                    out.append((a, b, c, int(xs)))
    return out


def test_monotone_flag_ties_are_monotone():
    """Section 4 prints strict inequalities, 0 < x_p < 3 dx: an extremum exactly on the stencil's
    outer edge leaves p monotone inside it, so the window is not flagged.  Just inside either edge
    it is flagged."""
    ties = _tie_windows()
    assert sum(1 for t in ties if t[3] == 0) > 20 and sum(1 for t in ties if t[3] == 3) > 20
    for a, b, c, _ in ties:
        assert O.monotone_flag(float(a), float(b), float(c)) == 0, (a, b, c)
    assert O.monotone_flag(0.0, 1.0, 3.0) == 0  # x_p = 0
    assert O.monotone_flag(3.0, 1.0, 0.0) == 0  # x_p = 3 dx
    assert O.monotone_flag(0.0, 1.0, 3.001) == 1  # x_p = 0.001/1.001: just above 0
    assert O.monotone_flag(3.001, 1.0, 0.0) == 1  # x_p = 3.002/1.001: just below 3 dx


def test_switch_leaves_eta_at_tie_windows():
    """Through the interface states: a line whose cells form x_p = 0 and x_p = 3 dx windows keeps
    the shape parameter at the interfaces next to them (switch on), like the switch-off line."""
    line = np.array([5.0, 4.0, 4.5, 0.0, 1.0, 3.0, 3.5, 3.0, 1.0, 0.0, 0.25, 0.5, 1.0, 1.5, 2.0, 2.5])
    # windows centred on cells 4 (0, 1, 3) and 8 (3, 1, 0) are the ties
    assert O.monotone_flag(*line[3:6]) == 0 and O.monotone_flag(*line[7:10]) == 0
    on = O.line_states(O.Problem(nx=line.size, flux=O.BURGERS), line)
    off = O.line_states(O.Problem(nx=line.size, flux=O.BURGERS, switch_mode=O.SWITCH_OFF), line)
    for cell in (4, 8):
        for iface in (cell, cell + 1):  # interfaces cell-1/2 and cell+1/2 (index i+1 for i+1/2)
            others = [q for q in (iface - 1, iface) if q != cell]  # the other adjacent cell
            if any(O.monotone_flag(*line[q - 1:q + 2]) for q in others):
                continue
            assert on[3][iface] == 0 and on[2][iface] == off[2][iface] != 0.0, (cell, iface)
            assert on[0][iface] == off[0][iface] and on[1][iface] == off[1][iface]


def test_monotone_flag_linear_and_constant_windows():
    assert O.monotone_flag(1.0, 2.0, 3.0) == 0  # linear: no extremum
    assert O.monotone_flag(0.5, 0.5, 0.5) == 0  # constant: 0/0
    assert O.monotone_flag(0.0, 1.0, 0.0) == 1  # peak in the middle cell
    assert O.monotone_flag(0.0, 0.0, 1.0) == 1  # quadratic through a step bottoms out inside


# ---------------------------------------------------------------------------------------
# Jiang-Shu smoothness indicators from their integral definition
# ---------------------------------------------------------------------------------------
def _beta_definition(u5):
    """beta_r = sum_{l=1,2} int_{I_i} h^{2l-1} (p_r^{(l)})^2 dx with p_r the quadratic whose
    cell averages on S_r(i) are the data (unit h, I_i = [0, 1]), in exact rationals."""
    u5 = [Fraction(x) for x in u5]
    out = []
    for r in range(3):
        cells = [-r + j for j in range(3)]  # cell offsets relative to i
        vals = [u5[2 + m] for m in cells]
        # p(x) = k0 + k1 x + k2 x^2 with average over [m, m+1] equal to vals
        M = [[Fraction(1), Fraction(2 * m + 1, 2), Fraction(3 * m * m + 3 * m + 1, 3)] for m in cells]
        # solve 3x3 by Cramer's rule
        def det(A):
            return (A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
                    - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
                    + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]))
        D = det(M)
        ks = []
        for col in range(3):
            Mc = [row[:] for row in M]
            for rr in range(3):
                Mc[rr][col] = vals[rr]
            ks.append(det(Mc) / D)
        k1, k2 = ks[1], ks[2]
        # int_0^1 (k1 + 2 k2 x)^2 dx + int_0^1 (2 k2)^2 dx
        first = k1 * k1 + 2 * k1 * k2 + Fraction(4, 3) * k2 * k2
        second = 4 * k2 * k2
        out.append(float(first + second))
    return out


def test_beta_matches_integral_definition():
    rng = np.random.default_rng(5)
    for _ in range(200):
        u5 = [int(v) for v in rng.integers(-9, 10, size=5)]
        got = O.beta(np.array(u5, dtype=float))
        np.testing.assert_allclose(got, _beta_definition(u5), rtol=1e-14, atol=1e-14)


def test_weno_reconstruction_exact_for_quadratics():
    """On quadratic data every substencil is exact, so the WENO value at the interface equals
    the quadratic's point value regardless of the nonlinear weights (eta = 0 there)."""
    # cell averages of x^2 on [m, m+1] are m^2 + m + 1/3; value of x^2 at x = 1 (right edge of cell 0)
    u5 = np.array([m * m + m + 1.0 / 3.0 for m in range(-2, 3)])
    assert O.recon_minus(u5, 0.0) == pytest.approx(1.0, abs=1e-12)
    assert O.recon_plus(u5, 0.0) == pytest.approx(0.0, abs=1e-12)


def test_quotient_free_switch_form_agrees_on_float_data():
    """The float-bulk kernels decide the Section 4 switch without forming the quotient: with
    p = u_i - u_{i-1} and q = u_{i+1} - u_i in double, the printed 0 < x_p < 3 holds exactly when
    p - q, 2p - q and p - 2q are non-zero with one sign (the sign of p - q against those of the
    other two, as two products).  On float data that equals the oracle's rounded-quotient test:
    random windows, windows with ties and near-ties planted, and windows spanning wide exponent
    ranges."""
    rng = np.random.default_rng(12)

    def quotient_free(a, b, c):
        p, q = b - a, c - b
        t1 = p - q
        t2, t3 = p + t1, t1 - q
        return int(t1 * t2 > 0.0 and t1 * t3 > 0.0)

    wins = [rng.standard_normal(3) for _ in range(20000)]
    wins += [rng.integers(-6, 7, 3).astype(float) * rng.choice([1e-3, 0.37, 1.0, 2.0 ** 40]) for _ in range(20000)]
    wins += [np.array([a, b, c], float) * s + o for a, b, c, _ in _tie_windows()
             for s in (1.0, 0.1, 3.7e5) for o in (0.0, 1.25, -1e3)]
    wins += [np.exp(rng.uniform(-80, 80, 3)) * rng.choice([-1.0, 1.0], 3) for _ in range(20000)]
    for w in wins:
        a, b, c = (float(np.float32(x)) for x in w)  # float data, widened exactly
        assert quotient_free(a, b, c) == O.monotone_flag(a, b, c), (a, b, c)
