"""Pins of the oracle's transverse Gauss-node collocation
(oracle.sldg_oracle.sweep_collocated).

* With one displacement for all nodes of a transverse cell, the collocated
  sweep is the plain sweep (the modal -> nodal -> modal round trip is the
  identity on polynomials of degree k, by the exactness of the o-point Gauss
  rule).
* The cell means sum to the same total (Gauss exactness for P_0).
* On the shear flow f_t + v f_x = 0, whose exact solution is f(x - v t, v),
  the cell-centre sweep (one displacement per transverse cell) is first
  order in h_v, while collocation converges at high order.
"""
import math

import numpy as np
import pytest

from oracle import sldg_oracle as O


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("dim,tdim", [(0, 1), (1, 0)])
def test_equal_node_shifts_reduce_to_the_plain_sweep(k, dim, tdim):
    rng = np.random.default_rng(10 * k + dim)
    ns = (12, 10)
    st = rng.standard_normal(((k + 1) ** 2, ns[0] * ns[1]))
    line = rng.uniform(-3, 3, ns[tdim])
    got = O.sweep_collocated(st, ns, k, dim, tdim, np.repeat(line[:, None], k + 1, axis=1))
    want = O.sweep(st, ns, k, dim, line, (tdim,))
    assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want))


def test_equal_node_shifts_in_three_dimensions():
    rng = np.random.default_rng(3)
    ns, k = (6, 5, 4), 2
    st = rng.standard_normal(((k + 1) ** 3, int(np.prod(ns))))
    line = rng.uniform(-2, 2, ns[2])
    got = O.sweep_collocated(st, ns, k, 1, 2, np.repeat(line[:, None], k + 1, axis=1))
    want = O.sweep(st, ns, k, 1, line, (2,))
    assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want))


def test_collocated_sweep_conserves_mass():
    rng = np.random.default_rng(4)
    ns, k = (16, 12), 3
    st = rng.standard_normal(((k + 1) ** 2, ns[0] * ns[1]))
    sig = rng.uniform(-3, 3, (ns[1], k + 1))
    out = O.sweep_collocated(st, ns, k, 0, 1, sig)
    assert abs(math.fsum(out[0].tolist()) - math.fsum(st[0].tolist())) <= 1e-14 * np.sum(np.abs(st[0]))


def _shear_error(nv, colloc, nx=64, k=2, T=1.0, nsteps=10):
    L = 2 * math.pi
    los, his = (0.0, -3.0), (L, 3.0)
    st = O.project_separable([(np.sin, lambda v: np.exp(-v * v / 2))], (nx, nv), los, his, k, nq=8)
    hx, hv, dt = L / nx, 6.0 / nv, T / nsteps
    xi, _ = O.gauss_legendre(k + 1)
    vc = -3.0 + (np.arange(nv) + 0.5) * hv
    for _ in range(nsteps):
        if colloc:
            st = O.sweep_collocated(st, (nx, nv), k, 0, 1,
                                    (vc[:, None] + 0.5 * hv * xi[None, :]) * dt / hx)
        else:
            st = O.sweep(st, (nx, nv), k, 0, vc * dt / hx, (1,))
    exact = [(np.sin, lambda v: np.cos(v * T) * np.exp(-v * v / 2)),
             (lambda x: -np.cos(x), lambda v: np.sin(v * T) * np.exp(-v * v / 2))]
    want = O.project_separable(exact, (nx, nv), los, his, k, nq=8)
    w = O.mode_weights(2, k)[:, None]
    return math.sqrt(np.sum(w * (st - want) ** 2) / np.sum(w * want ** 2))


def test_collocation_is_high_order_in_the_transverse_cell_size():
    c8, c16 = _shear_error(8, True), _shear_error(16, True)
    r8, r16 = _shear_error(8, False), _shear_error(16, False)
    assert r8 / r16 < 2.5                     # cell centres: first order
    assert c8 / c16 > 8.0                     # collocation: third order or better
    assert c16 < r16 / 100
