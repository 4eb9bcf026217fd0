"""The seeded input generators: exact cell averages checked by quadrature."""
import math

import numpy as np
from scipy import integrate

from paper_1602_00182_amd import inputs as I


def test_advection2d_cell_averages_match_quadrature():
    n = 8
    h = 1.0 / n
    u = I.advection2d_sine(n).u0.reshape(n, n)  # [j, i]
    for j, i in [(0, 0), (3, 5), (7, 2), (6, 6)]:
        v, _ = integrate.dblquad(lambda y, x: math.sin(2 * math.pi * (x + y)), i * h, (i + 1) * h,
                                 lambda x: j * h, lambda x: (j + 1) * h, epsabs=1e-14, epsrel=1e-14)
        assert abs(u[j, i] - v / (h * h)) < 1e-13


def test_sine_cell_averages_match_quadrature():
    n = 10
    u = I.sine_cell_averages(n)
    h = 2.0 / n
    for i in (0, 4, 9):
        a = -1.0 + i * h
        v, _ = integrate.quad(lambda x: math.sin(math.pi * x), a, a + h, epsabs=1e-15)
        assert abs(u[i] - v / h) < 1e-14
