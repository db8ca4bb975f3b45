"""Pins of the oracle's FP16 storage with per-plane power-of-two scaling.

The scaling policy is this library's design, not the paper's: the paper's
precision axis is FP64 and FP32 storage of the coefficients with the leading
ones in FP64 (section II-A, section III-A).  Its purpose is a property of
FP16 (a narrow exponent range).  These tests pin the oracle's emulation of
the policy against things the oracle's code does not compute itself:

* numpy's float16 cast, an independent round-to-nearest-even;
* the defining interval of the storage exponent, checked with exact
  power-of-two arithmetic;
* exact invariance under scaling the state by a power of two, which plain
  FP16 storage does not have;
* the repair of a plane that grows beyond its headroom in one sweep.
"""
import math

import numpy as np
import pytest

from oracle import sldg_oracle as O
from paper_1603_07008_amd import inputs


def f16(x):
    """numpy's float16 cast (RNE), back in FP64."""
    with np.errstate(over="ignore"):
        return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)


def _vlasov_2d(nx=64, nv=48, steps=1):
    prob = inputs.vlasov_2d(nx=nx, nv=nv, steps=steps)
    st = O.project_separable(prob.f0_terms, prob.ns, prob.los, prob.his, prob.k)
    seq = [(s.dim, s.sigma, s.dep) for s in prob.seq]
    return prob, st, seq


@pytest.mark.parametrize("h", [0, 4, 8, 14])
def test_storage_exponent_interval(h):
    rng = np.random.default_rng(h)
    amax = np.float32(10.0) ** rng.uniform(-30, 30, 2000).astype(np.float32)
    amax = np.concatenate([amax, np.float32(2.0) ** np.arange(-60, 60, dtype=np.float32)])
    for a in amax.astype(np.float64):
        e = O.storage_exponent(a, h)
        if O.SCALE_EMIN < e < O.SCALE_EMAX:
            lo, hi = 2.0 ** (14 - h), 2.0 ** (15 - h)
            v = math.ldexp(a, e)                      # exact
            assert lo <= v < hi, (a, h, e, v)
    for bad in (0.0, float("inf"), float("nan")):
        assert O.storage_exponent(bad, h) is None


@pytest.mark.parametrize("unit", [1.0, 2.0 ** -40, 2.0 ** 20])
def test_to_scaled_is_rne_at_the_plane_exponent(unit):
    prob, st, _ = _vlasov_2d()
    st = st * unit
    vals, e, amax = O.to_scaled(st, prob.k, prob.ndim)
    assert np.array_equal(vals[0], st[0]) and e[0] == 0          # the FP64 mass mode
    for m in range(1, st.shape[0]):
        stored = np.ldexp(vals[m], int(e[m]))
        assert np.array_equal(stored, f16(np.ldexp(st[m], int(e[m])))), m
        assert np.all(np.isfinite(stored)) and np.max(np.abs(stored)) <= 65504.0
        assert amax[m] == float(np.float32(np.max(np.abs(st[m]))))
        v = math.ldexp(amax[m], int(e[m]))
        assert 2.0 ** (14 - O.SCALE_HEADROOM) <= v < 2.0 ** (15 - O.SCALE_HEADROOM)


def test_sweep_scaled_rounds_the_exact_update():
    prob, st, seq = _vlasov_2d()
    cur = O.to_scaled(st, prob.k, prob.ndim)
    for dim, sig, dep in seq * 3:
        vals, e_in, a_in = cur
        acc = O.sweep(vals, prob.ns, prob.k, dim, sig, dep, "fp64")
        cur = O.sweep_scaled(vals, e_in, a_in, prob.ns, prob.k, dim, sig, dep)
        out, e_out, a_out = cur
        assert np.array_equal(out[0], acc[0])
        for m in range(1, out.shape[0]):
            assert a_out[m] == float(np.float32(np.max(np.abs(acc[m]))))
            pred = O.storage_exponent(a_in[m], O.SCALE_HEADROOM)
            grew = math.ldexp(a_out[m], pred) >= 2.0 ** 15
            want_e = O.storage_exponent(a_out[m], O.SCALE_REPAIR_HEADROOM) if grew else pred
            assert e_out[m] == want_e, m
            stored = np.ldexp(out[m], int(e_out[m]))
            assert np.array_equal(stored, f16(np.ldexp(acc[m], int(e_out[m])))), m
            assert np.max(np.abs(stored)) < 2.0 ** 15


def test_power_of_two_invariance_which_plain_fp16_lacks():
    prob, st, seq = _vlasov_2d()
    t = -40
    a = O.run_sequence_scaled(O.to_scaled(st, prob.k, prob.ndim), prob.ns, prob.k, seq, steps=3)
    b = O.run_sequence_scaled(O.to_scaled(np.ldexp(st, t), prob.k, prob.ndim), prob.ns, prob.k,
                              seq, steps=3)
    assert np.array_equal(b[0], np.ldexp(a[0], t))
    assert np.array_equal(b[1][1:], a[1][1:] - t)
    # plain FP16 storage of the same small state flushes the higher modes
    plain = O.run_sequence(O.to_tier(np.ldexp(st, t), "fp16"), prob.ns, prob.k, seq, "fp16", 3)
    assert np.all(plain[1:] == 0.0)
    assert np.any(a[0][1:] != 0.0)


def test_repair_of_a_plane_that_outgrows_its_headroom():
    # 1D, k = 2: a step in the cell means and tiny higher modes; one sweep by a
    # fraction of a cell creates O(0.1) quadratic modes at the step, far beyond
    # the exponent predicted from the tiny input
    n, k = 16, 2
    rng = np.random.default_rng(3)
    st = np.zeros((3, n))
    st[0, : n // 2] = 1.0
    st[1:] = 1e-12 * rng.standard_normal((2, n))
    vals, e, amax = O.to_scaled(st, k, 1)
    out, e_out, a_out = O.sweep_scaled(vals, e, amax, (n,), k, 0, 0.3)
    acc = O.sweep(vals, (n,), k, 0, 0.3, (), "fp64")
    for m in (1, 2):
        pred = O.storage_exponent(amax[m], O.SCALE_HEADROOM)
        assert math.ldexp(a_out[m], pred) >= 2.0 ** 15          # the repair case
        assert e_out[m] == O.storage_exponent(a_out[m], O.SCALE_REPAIR_HEADROOM)
        stored = np.ldexp(out[m], int(e_out[m]))
        assert np.all(np.isfinite(stored))
        assert np.array_equal(stored, f16(np.ldexp(acc[m], int(e_out[m]))))


def test_scaled_fp16_run_accuracy_and_mass():
    prob, st, seq = _vlasov_2d(steps=20)
    ref = O.run_sequence(st, prob.ns, prob.k, seq, "fp64", prob.steps)
    out, _, _ = O.run_sequence_scaled(O.to_scaled(st, prob.k, prob.ndim), prob.ns, prob.k, seq,
                                      prob.steps)
    w = O.mode_weights(prob.ndim, prob.k)[:, None]
    rel = math.sqrt(np.sum(w * (out - ref) ** 2) / np.sum(w * ref ** 2))
    assert rel < 5e-3
    m0, m1 = O.mass_sum(st[0]), O.mass_sum(out[0])
    assert abs(m1 - m0) <= 1e-14 * abs(m0)
