"""Regression test for the plan's two scratch buffers (the absmax partials of
scaled FP16 storage and the field-solve scratch): each is grown and freed by
its own helper only.  A field solve, then scaled calls that grow the partial
buffer, then the field solve again must still match the oracle, and the plan
must be destroyed cleanly afterwards.

Field parity: both sides compute in FP64 from the same stored values (section
II, the field E(x) that drives the v-sweep), so they agree to 1e-12 of the
largest field value.  Scaled sweeps: exponents exactly, values within the
FP16 bound at the plane's scale (section II-A update rule)."""
import numpy as np
import pytest

from oracle import sldg_oracle as O
from paper_1603_07008_amd import inputs
from gpu_helpers import have_gpu, upload_nd
from test_gpu_scaled import _check_sweep, _dev, download_scaled, upload_scaled

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sl():
    if not have_gpu():
        pytest.skip("no HIP device")
    import paper_1603_07008_amd as sl
    sl.lib()
    return sl


def _field_1d(sl, plan, st, ns, k):
    import torch
    hx, hv, dt = 0.37, 0.21, 0.1
    m, h = upload_nd(st, plan)
    field = torch.empty(ns[0], dtype=torch.float64, device="cuda")
    plan.poisson_shift(m, h, hx, hv, dt, field_out=field)
    want = O.poisson_field(st, ns, k, hx, hv)
    got = field.cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-12 * float(np.max(np.abs(want)))


def _field_2d(sl, plan, st, ns):
    import torch
    h = (0.37, 0.29, 0.21, 0.17)
    m, hi = upload_nd(st, plan)
    nxx = ns[0] * ns[1]
    field = torch.empty(2 * nxx, dtype=torch.float64, device="cuda")
    plan.poisson_shift_2d(m, hi, h, 0.1, field_out=field)
    W1, W2 = O.poisson_field_2d(st, ns, h)
    got = field.cpu().numpy()
    scale = max(np.max(np.abs(W1)), np.max(np.abs(W2)))
    assert np.max(np.abs(got[:nxx] - W1)) <= 1e-12 * scale
    assert np.max(np.abs(got[nxx:] - W2)) <= 1e-12 * scale


def _scaled_calls(sl, plan, st, ns, k, dim, dep, seed):
    """A scaled import (grows the partials to n_hi x 256 slots) and one
    scaled sweep, checked against the oracle."""
    import torch
    ndim = len(ns)
    scaled = O.to_scaled(st, k, ndim)
    hi = torch.empty((plan.n_hi, plan.cells), dtype=torch.float16, device="cuda")
    sc = plan.empty_scale()
    plan.scaled_import(_dev(st[1:]), hi, sc)
    got_imp = download_scaled(plan, _dev(st[0]), hi, sc)
    assert np.array_equal(got_imp[1], scaled[1]) and np.array_equal(got_imp[0], scaled[0])
    rng = np.random.default_rng(seed)
    ntab = int(np.prod([ns[e] for e in dep]))
    sigma = rng.uniform(-2.0, 2.0, ntab)
    want = O.sweep_scaled(*scaled, ns, k, dim, sigma, dep)
    mag = O.sweep(scaled[0], ns, k, dim, sigma, dep, absolute=True)
    m_in, h_in, s_in = upload_scaled(plan, scaled)
    m_out, h_out = plan.empty_state()
    s_out = plan.empty_scale()
    plan.advect_dim_scaled(dim, _dev(sigma), sum(1 << e for e in dep), m_in, h_in, s_in,
                           m_out, h_out, s_out)
    got = download_scaled(plan, m_out, h_out, s_out)
    _check_sweep(got, want, mag, O.fp64_modes(ndim, k).astype(bool), k, f"{ns} dim {dim}")


@pytest.mark.parametrize("ns,k", [((40, 24), 2), ((33, 17), 1)])
def test_field_solve_then_scaled_growth_then_field_solve_xv(sl, ns, k):
    import torch
    st = O.to_tier(inputs.random_coefficients(2, k, ns[0] * ns[1], seed=31 + k), "fp16")
    plan = sl.Plan(ns, k, "fp16")
    _field_1d(sl, plan, st, ns, k)
    _scaled_calls(sl, plan, inputs.random_coefficients(2, k, ns[0] * ns[1], seed=41), ns, k,
                  1, (0,), 5)
    _field_1d(sl, plan, st, ns, k)
    torch.cuda.synchronize()
    plan.close()


def test_field_solve_then_scaled_growth_then_field_solve_4d(sl):
    import torch
    ns, k = (8, 6, 5, 4), 1
    cells = int(np.prod(ns))
    st = O.to_tier(inputs.random_coefficients(4, k, cells, seed=51), "fp16")
    plan = sl.Plan(ns, k, "fp16")
    _field_2d(sl, plan, st, ns)
    _scaled_calls(sl, plan, inputs.random_coefficients(4, k, cells, seed=52), ns, k, 2,
                  (0, 1), 6)
    _field_2d(sl, plan, st, ns)
    _scaled_calls(sl, plan, inputs.random_coefficients(4, k, cells, seed=53), ns, k, 0,
                  (2,), 7)
    _field_2d(sl, plan, st, ns)
    torch.cuda.synchronize()
    plan.close()
