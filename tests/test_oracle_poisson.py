"""Pins of the oracle's self-consistent field for 1D-1V problems
(oracle.sldg_oracle.poisson_field / poisson_shift).

The paper states the Vlasov equation with a given field (section II) and no
field equation; the reading taken (Gauss's law dE/dx = rho - mean(rho), zero
mean, in the paper's +E d_v f sign convention) is pinned by:

* the closed form for rho = (1 + eps cos(kappa x)) int M dv: E = (eps/kappa)
  sin(kappa x), and its convergence under refinement;
* an independent route: Gauss quadrature of the reconstructed piecewise
  density from the left boundary to every point, the zero-mean constant from
  the quadrature of E itself;
* physics: linear Landau damping of the field for kappa = 0.5 (the textbook
  values of linear theory, damping rate -0.1533 and frequency 1.4156), with
  the whole Strang split step X(dt/2) V(dt) X(dt/2) driven by the field.
"""
import math

import numpy as np
import pytest

from oracle import sldg_oracle as O
from paper_1603_07008_amd import inputs


def _landau_state(nx, nv, k, kappa=0.5, eps=0.01, vmax=6.0):
    L = 2 * math.pi / kappa
    ns, los, his = (nx, nv), (0.0, -vmax), (L, vmax)
    st = O.project_separable([(lambda x: 1 + eps * np.cos(kappa * x), inputs.maxwellian)],
                             ns, los, his, k)
    return st, ns, L / nx, 2 * vmax / nv


def test_field_matches_closed_form_and_converges():
    kappa, eps = 0.5, 0.01
    errs = []
    for nx in (32, 64):
        st, ns, hx, hv = _landau_state(nx, 96, 2)
        E = O.poisson_field(st, ns, 2, hx, hv)
        xc = (np.arange(nx) + 0.5) * hx
        errs.append(float(np.max(np.abs(E - eps / kappa * np.sin(kappa * xc)))))
    assert errs[0] < 3e-8 and errs[1] < errs[0] / 8, errs


def test_field_has_zero_mean_and_is_linear_in_the_state():
    st, ns, hx, hv = _landau_state(40, 48, 3)
    E = O.poisson_field(st, ns, 3, hx, hv)
    assert abs(math.fsum(E.tolist())) <= 1e-15 * float(np.sum(np.abs(E)))
    rng = np.random.default_rng(2)
    pert = 1e-3 * rng.standard_normal(st.shape)
    E2 = O.poisson_field(st + pert, ns, 3, hx, hv)
    Ep = O.poisson_field(pert, ns, 3, hx, hv)
    assert np.allclose(E2, E + Ep, rtol=0, atol=1e-15)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_field_against_quadrature_of_the_density(k):
    nx, nv = 12, 10
    rng = np.random.default_rng(k)
    st = rng.standard_normal(((k + 1) ** 2, nx * nv))
    hx, hv = 0.7, 0.3
    ns = (nx, nv)
    E = O.poisson_field(st, ns, k, hx, hv)
    # the density as a piecewise polynomial in x, from the state directly
    o = k + 1
    r = np.zeros((o, nx))
    for j in range(o):
        r[j] = hv * st[j].reshape(nv, nx).sum(axis=0)
    L = nx * hx
    xg, wg = np.polynomial.legendre.leggauss(k + 3)

    def integral(a, b):          # int_a^b rho(x) dx within one cell, Gauss rule
        x = 0.5 * (a + b) + 0.5 * (b - a) * xg
        return 0.5 * (b - a) * float(np.sum(wg * O.eval_1d(r, nx, 0.0, L, x)))

    rbar = sum(integral(i * hx, (i + 1) * hx) for i in range(nx)) / L

    def E0(x):                   # antiderivative of rho - rbar from 0
        i = min(int(x // hx), nx - 1)
        return (sum(integral(c * hx, (c + 1) * hx) for c in range(i))
                + integral(i * hx, x) - rbar * x)

    mean = sum(0.5 * hx * wq * E0(i * hx + 0.5 * hx * (xq + 1)) for i in range(nx)
               for xq, wq in zip(xg, wg)) / L
    want = np.array([E0((i + 0.5) * hx) - mean for i in range(nx)])
    assert np.allclose(E, want, rtol=0, atol=1e-12 * float(np.max(np.abs(want)))), \
        float(np.max(np.abs(E - want)))


def test_landau_damping_rate_and_frequency():
    nx, nv, k, dt = 32, 64, 2, 0.1
    st, ns, hx, hv = _landau_state(nx, nv, k)
    vc = -6.0 + (np.arange(nv) + 0.5) * hv
    sx = vc * (0.5 * dt) / hx
    ts, logE = [], []
    for n in range(230):
        E = O.poisson_field(st, ns, k, hx, hv)
        ts.append(n * dt)
        logE.append(0.5 * math.log(float(np.sum(E * E)) * hx))
        st = O.sweep(st, ns, k, 0, sx, (1,))
        st = O.sweep(st, ns, k, 1, O.poisson_shift(st, ns, k, hx, hv, dt), (0,))
        st = O.sweep(st, ns, k, 0, sx, (1,))
    ts, logE = np.array(ts), np.array(logE)
    peaks = [i for i in range(1, len(ts) - 1)
             if logE[i] > logE[i - 1] and logE[i] > logE[i + 1] and 1.0 < ts[i] < 22.0]
    gamma = np.polyfit(ts[peaks], logE[peaks], 1)[0]
    omega = math.pi / float(np.mean(np.diff(ts[peaks])))     # |E| peaks twice per period
    assert abs(gamma - (-0.1533)) < 0.03 * 0.1533, gamma
    assert abs(omega - 1.4156) < 0.03 * 1.4156, omega
