"""Pins of the oracle's characteristic-wise Euler reconstruction (Roe-averaged eigen-system),
checked against what the Euler flux of Example 4 (and its 2D form) fixes by itself:

* left and right eigenvector matrices are inverse to each other;
* R diag(lambda) L is the Jacobian of the flux (complex-step derivative of the flux formula) at
  the state with the returned eigenvalues' velocity and sound speed;
* Roe's property: R diag(lambda) L (U_R - U_L) = F(U_R) - F(U_L) exactly (up to rounding);
* uniform states stay uniform, the cell-average sums are conserved;
* on Sod's problem against the exact Riemann solution: the density's total variation falls to
  the exact value (component-wise reconstruction overshoots it) at no loss of L1 accuracy;
* design order on a smooth density wave.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_1602_00182_amd import inputs as I

sys.path.insert(0, __file__.rsplit("/", 1)[0])
import exact_riemann as ER  # noqa: E402

G = 1.4


def _flux(U, direction):
    """Euler flux of conservative U (1D: rho, m, E; 2D: rho, mx, my, E), complex-safe."""
    if len(U) == 3:
        rho, m, E = U
        u = m / rho
        p = (G - 1.0) * (E - 0.5 * rho * u * u)
        return np.array([m, m * u + p, (E + p) * u])
    rho, mx, my, E = U
    u, v = mx / rho, my / rho
    p = (G - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    if direction == 0:
        return np.array([mx, mx * u + p, my * u, (E + p) * u])
    return np.array([my, mx * v, my * v + p, (E + p) * v])


def _jacobian(U, direction):
    m = len(U)
    J = np.zeros((m, m))
    h = 1e-30
    for k in range(m):
        Uc = np.array(U, dtype=complex)
        Uc[k] += 1j * h
        J[:, k] = np.imag(_flux(Uc, direction)) / h
    return J


def _random_state(rng, m):
    rho = rng.uniform(0.1, 2.0)
    u = rng.uniform(-2.0, 2.0)
    v = rng.uniform(-2.0, 2.0)
    p = rng.uniform(0.1, 2.0)
    if m == 3:
        return np.array([rho, rho * u, p / (G - 1.0) + 0.5 * rho * u * u])
    return np.array([rho, rho * u, rho * v, p / (G - 1.0) + 0.5 * rho * (u * u + v * v)])


CASES = [(3, 0), (4, 0), (4, 1)]


@pytest.mark.parametrize("m,direction", CASES)
def test_eigenvectors_are_inverse(m, direction):
    rng = np.random.default_rng(10 + m + direction)
    pb = O.Problem(nx=8, flux=O.EULER, ncomp=m, dim=1 if m == 3 else 2, ny=8, charwise=1)
    for _ in range(50):
        Lm, Rm, lam = O.char_basis(pb, direction, _random_state(rng, m), _random_state(rng, m))
        assert np.max(np.abs(Lm @ Rm - np.eye(m))) <= 1e-12
        assert lam[0] < lam[1] <= lam[-2] < lam[-1]


@pytest.mark.parametrize("m,direction", CASES)
def test_eigen_system_is_the_flux_jacobian(m, direction):
    """R diag(lam) L equals dF/dU at the state with normal velocity lam[1] and sound speed
    (lam[-1] - lam[0]) / 2 (any density; the tangential velocity from Roe's property below)."""
    rng = np.random.default_rng(20 + m + direction)
    pb = O.Problem(nx=8, flux=O.EULER, ncomp=m, dim=1 if m == 3 else 2, ny=8, charwise=1)
    for _ in range(20):
        UL, UR = _random_state(rng, m), _random_state(rng, m)
        Lm, Rm, lam = O.char_basis(pb, direction, UL, UR)
        A = Rm @ np.diag(lam) @ Lm
        c = 0.5 * (lam[-1] - lam[0])
        un = lam[1]
        if m == 3:
            u, v = un, 0.0
        else:
            # the tangential velocity is the one entry of the shear eigenvector that is not 0/1
            t = Rm[3, 2]
            u, v = (un, t) if direction == 0 else (t, un)
        H = c * c / (G - 1.0) + 0.5 * (u * u + v * v)
        rho = 0.7
        E = rho * (H + (G - 1.0) * 0.5 * (u * u + v * v)) / G
        U = np.array([rho, rho * u, E]) if m == 3 else np.array([rho, rho * u, rho * v, E])
        J = _jacobian(U, direction)
        assert np.max(np.abs(A - J)) <= 1e-11 * max(1.0, np.max(np.abs(J)))


@pytest.mark.parametrize("m,direction", CASES)
def test_roe_property(m, direction):
    rng = np.random.default_rng(30 + m + direction)
    pb = O.Problem(nx=8, flux=O.EULER, ncomp=m, dim=1 if m == 3 else 2, ny=8, charwise=1)
    for _ in range(50):
        UL, UR = _random_state(rng, m), _random_state(rng, m)
        Lm, Rm, lam = O.char_basis(pb, direction, UL, UR)
        lhs = Rm @ np.diag(lam) @ Lm @ (UR - UL)
        rhs = _flux(UR, direction) - _flux(UL, direction)
        assert np.max(np.abs(lhs - rhs)) <= 1e-12 * max(1.0, np.max(np.abs(rhs)))


def test_nonphysical_state_is_rejected():
    pb = O.Problem(nx=8, flux=O.EULER, ncomp=3, charwise=1)
    with pytest.raises(O.OracleError):
        O.char_basis(pb, 0, [1.0, 0.0, -1.0], [1.0, 0.0, 2.5])


def test_charwise_needs_euler():
    pb = O.Problem(nx=8, flux=O.BURGERS, charwise=1)
    with pytest.raises(O.OracleError):
        O.rhs(pb, np.zeros(8))


@pytest.mark.parametrize("recon", [O.RBF_WENO5, O.RBF_ENO3, O.RBF_WENO3, O.ENO2])
def test_uniform_state_and_conservation(recon):
    n = 40
    rng = np.random.default_rng(5)
    pb = O.Problem(nx=n, flux=O.EULER, ncomp=3, bc=O.PERIODIC, recon=recon, charwise=1)
    U = _random_state(rng, 3)
    u = np.repeat(U, n)
    L, _ = O.rhs(pb, u)
    assert np.max(np.abs(L)) <= 1e-10  # rounding of the projections only, amplified by 1/dx = 20
    w = I.euler_riemann_batch(count=1, seed=8, nmin=n, nmax=n)[0]
    pb2 = O.Problem(nx=n, flux=O.EULER, ncomp=3, bc=O.PERIODIC, recon=recon, charwise=1)
    u1, _, _ = O.solve(pb2, w.u0, 0.05)
    m0 = w.u0.reshape(3, n).sum(axis=1)
    m1 = u1.reshape(3, n).sum(axis=1)
    assert np.max(np.abs(m1 - m0) / np.abs(m0)) <= 1e-13


def _tv(x):
    return float(np.sum(np.abs(np.diff(x))))


@pytest.mark.parametrize("recon", [O.RBF_WENO5, O.RBF_ENO3, O.RBF_WENO3, O.RBF_ENO2])
def test_sod_characteristic_removes_overshoots(recon):
    """Sod at the paper's settings (Example 4: N = 600 would do; N = 200 is enough here, CFL
    0.1, T = 0.2): the exact density has total variation 0.875."""
    n = 200
    w = I.sod(n, cfl=0.1)
    exact = ER.density_cell_averages(n, 0.2, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    out = {}
    for cw in (0, 1):
        pb = O.Problem(nx=n, flux=O.EULER, ncomp=3, bc=O.TRANSMISSIVE, cfl=0.1, recon=recon, charwise=cw)
        u, t, _ = O.solve(pb, w.u0, 0.2)
        rho = u[:n]
        out[cw] = (float(np.mean(np.abs(rho - exact))), _tv(rho))
    assert _tv(exact) == pytest.approx(0.875, abs=1e-12)
    assert out[0][1] > 0.875 * 1.02  # component-wise: overshoots
    assert out[1][1] <= 0.875 * 1.005  # characteristic-wise: essentially non-oscillatory
    assert out[1][0] <= 1.05 * out[0][0]


def test_smooth_density_wave_design_order():
    """rho = 1 + 0.2 sin(pi x), u = 1, p = 1 (periodic) is translated exactly; RBF-WENO5 with
    characteristic reconstruction converges at fifth order (dt small enough to hide RK3)."""
    errs = []
    for n in (20, 40):
        h = 2.0 / n
        rho = 1.0 + 0.2 * I.sine_cell_averages(n)
        U = I.euler_prim_to_cons(rho, np.ones(n), np.ones(n)).reshape(-1)
        pb = O.Problem(nx=n, flux=O.EULER, ncomp=3, bc=O.PERIODIC, recon=O.RBF_WENO5,
                       switch_mode=O.SWITCH_OFF, charwise=1, dt_fixed=0.02 * h)
        u, t, _ = O.solve(pb, U, 0.2)
        exact = 1.0 + 0.2 * I.sine_cell_averages(n, phase=-0.2 * math.pi)
        errs.append(float(np.mean(np.abs(u[:n] - exact))))
    order = math.log2(errs[0] / errs[1])
    assert order > 4.5, errs
