"""Pins of the oracle's self-consistent field of (x1, x2, v1, v2) problems
(oracle.sldg_oracle.poisson_field_2d, density_means_2d).

Gauss's law div E = rho - mean(rho), E = -grad phi periodic, has for the
density rho = 1 + sum_w a_w cos(kappa_w . x + phi_w) the field
E = sum_w a_w kappa_w sin(kappa_w . x + phi_w) / |kappa_w|^2.  The states
below carry such densities exactly (up to the projection's quadrature
rounding), on grids with N1 != N2 and L1 != L2, with wave vectors that are
not symmetric in x1 and x2: a swapped axis, a sign, a missing cell-average
factor or a wrong normalisation each fails one of them.
"""
import math

import numpy as np
import pytest

from oracle import sldg_oracle as O

NS = (12, 10, 3, 2)
L1, L2 = 4.0 * math.pi, 3.0 * math.pi
LV = 12.0
LOS = (0.0, 0.0, -6.0, -6.0)
HIS = (L1, L2, 6.0, 6.0)
H = (L1 / NS[0], L2 / NS[1], LV / NS[2], LV / NS[3])


def _flat_v(v):
    return np.full_like(np.asarray(v, dtype=np.float64), 1.0 / LV)


def _wave_terms(a, p1, p2, phi):
    """a cos(kappa . x + phi) / LV^2 as two separable terms."""
    k1, k2 = 2 * math.pi * p1 / L1, 2 * math.pi * p2 / L2
    return [(lambda x, k1=k1: a * np.cos(k1 * x + phi), lambda y, k2=k2: np.cos(k2 * y), _flat_v, _flat_v),
            (lambda x, k1=k1: -a * np.sin(k1 * x + phi), lambda y, k2=k2: np.sin(k2 * y), _flat_v, _flat_v)]


def _state(waves, k=2, background=1.0):
    terms = [(lambda x: np.full_like(x, background), lambda y: np.ones_like(y), _flat_v, _flat_v)]
    for w in waves:
        terms += _wave_terms(*w)
    return O.project_separable(terms, NS, LOS, HIS, k, nq=8)


def _exact(waves):
    x1 = (np.arange(NS[0]) + 0.5) * H[0]
    x2 = (np.arange(NS[1]) + 0.5) * H[1]
    X1, X2 = np.meshgrid(x1, x2)                       # [N2, N1], x1 fastest
    E1, E2 = np.zeros_like(X1), np.zeros_like(X1)
    for a, p1, p2, phi in waves:
        k1, k2 = 2 * math.pi * p1 / L1, 2 * math.pi * p2 / L2
        s = a * np.sin(k1 * X1 + k2 * X2 + phi) / (k1 * k1 + k2 * k2)
        E1 += k1 * s
        E2 += k2 * s
    return E1.ravel(), E2.ravel()


WAVES = [
    [(0.01, 1, 0, 0.0)],
    [(0.02, 0, 2, 0.3)],
    [(0.01, 1, 1, -0.7)],
    [(0.03, -2, 1, 1.1), (0.01, 3, 0, 0.2), (0.02, 1, -3, 2.5)],
]


@pytest.mark.parametrize("waves", WAVES)
def test_field_of_resolved_waves_is_exact(waves):
    E1, E2 = O.poisson_field_2d(_state(waves), NS, H)
    W1, W2 = _exact(waves)
    scale = max(np.max(np.abs(W1)), np.max(np.abs(W2)))
    assert np.max(np.abs(E1 - W1)) <= 1e-13 * scale
    assert np.max(np.abs(E2 - W2)) <= 1e-13 * scale


def test_shift_is_field_times_dt_over_hv():
    waves = WAVES[3]
    st = _state(waves)
    E1, E2 = O.poisson_field_2d(st, NS, H)
    s1, s2 = O.poisson_shift_2d(st, NS, H, 0.1)
    assert np.array_equal(s1, E1 * 0.1 / H[2]) and np.array_equal(s2, E2 * 0.1 / H[3])


def test_x2_independent_density_has_no_x2_field():
    E1, E2 = O.poisson_field_2d(_state([(0.05, 2, 0, 0.4)]), NS, H)
    assert np.max(np.abs(E2)) <= 1e-16 and np.max(np.abs(E1)) > 1e-3


def test_field_has_zero_mean_and_ignores_a_constant_density():
    waves = WAVES[3]
    E1, E2 = O.poisson_field_2d(_state(waves), NS, H)
    F1, F2 = O.poisson_field_2d(_state(waves, background=7.5), NS, H)
    assert abs(math.fsum(E1.tolist())) <= 1e-16 * E1.size and abs(math.fsum(E2.tolist())) <= 1e-16 * E2.size
    assert np.max(np.abs(E1 - F1)) <= 1e-14 and np.max(np.abs(E2 - F2)) <= 1e-14


def test_nyquist_density_gives_no_field():
    # sin(pi x1 / h1): cell means alternate in sign, the Nyquist mode of x1
    terms = [(lambda x: np.sin(math.pi * x / H[0]), lambda y: np.ones_like(y), _flat_v, _flat_v)]
    st = O.project_separable(terms, NS, LOS, HIS, 1, nq=8)
    rho = O.density_means_2d(st, NS, H[2], H[3])
    assert np.max(np.abs(rho)) > 0.5
    E1, E2 = O.poisson_field_2d(st, NS, H)
    assert np.max(np.abs(E1)) <= 1e-15 and np.max(np.abs(E2)) <= 1e-15


def test_density_integrates_the_velocity_profile():
    # f = (1 + 0.1 cos x1 cos(2 pi x2 / L2)) M(v1) M(v2): the x cell means of
    # rho are the x cell means of the x factor times erf(6 / sqrt 2)^2
    ns = (8, 6, 10, 12)
    h = (L1 / 8, L2 / 6, LV / 10, LV / 12)
    M = lambda v: np.exp(-v * v / 2) / math.sqrt(2 * math.pi)
    terms = [(lambda x: np.ones_like(x), lambda y: np.ones_like(y), M, M),
             (lambda x: 0.1 * np.cos(2 * math.pi * x / L1), lambda y: np.cos(2 * math.pi * y / L2), M, M)]
    st = O.project_separable(terms, ns, LOS, HIS, 1, nq=10)
    rho = O.density_means_2d(st, ns, h[2], h[3])
    vint = math.erf(6 / math.sqrt(2)) ** 2
    c1 = (np.arange(8) + 0.5) * h[0]
    c2 = (np.arange(6) + 0.5) * h[1]
    sinc = lambda z: math.sin(z) / z
    g = 1 + 0.1 * np.outer(np.cos(2 * math.pi * c2 / L2) * sinc(math.pi / 6),
                           np.cos(2 * math.pi * c1 / L1) * sinc(math.pi / 8))
    assert np.max(np.abs(rho - vint * g)) <= 1e-11
