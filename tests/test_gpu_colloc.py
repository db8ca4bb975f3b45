"""GPU parity of the transverse Gauss-node collocated sweep
(sldg_advect_dim_collocated) against the oracle's sweep_collocated, on the
same seeded inputs; reduction to the plain sweep, mass, and the accuracy gain
on a shear flow, on the GPU.

Element bound: both sides compute in FP64 (in different orders) and round
the narrow modes to nearest even, so they agree to one storage-format ulp
plus an FP64 accumulation error."""
import math

import numpy as np
import pytest

from oracle import sldg_oracle as O
from paper_1603_07008_amd import inputs
from gpu_helpers import download, download_nd, have_gpu, ulp, upload, upload_nd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sl():
    if not have_gpu():
        pytest.skip("no HIP device")
    import paper_1603_07008_amd as sl
    sl.lib()
    return sl


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


CASES = [
    # ns, k, dim, tdim, ndouble
    ((24, 16), 2, 0, 1, 1),
    ((24, 16), 2, 1, 0, 1),
    ((17, 9), 1, 0, 1, 1),
    ((13, 11), 3, 1, 0, 1),
    ((8, 6, 5), 2, 0, 2, 1),
    ((8, 6, 5), 1, 2, 1, 1),
    ((20, 12), 2, 0, 1, 2),
    # transverse stride a multiple of 64 cells (one transverse cell per wave)
    ((64, 12), 2, 0, 1, 1),
    ((16, 8, 6), 1, 1, 2, 1),
    ((64, 10), 3, 0, 1, 2),
    ((8, 8, 3, 4), 2, 0, 2, 1),
    ((4, 16, 4, 5), 2, 3, 2, 2),
]


@pytest.mark.parametrize("ns,k,dim,tdim,ndouble", CASES)
@pytest.mark.parametrize("tier", ["fp64", "fp32", "bf16"])
def test_collocated_sweep_matches_oracle(sl, ns, k, dim, tdim, ndouble, tier):
    ndim = len(ns)
    st = inputs.random_coefficients(ndim, k, int(np.prod(ns)), seed=sum(ns) + k)
    st = O.to_tier(st, tier, ndouble, k, ndim)
    rng = np.random.default_rng(k + 7 * dim)
    sig = rng.uniform(-4.0, 4.0, (ns[tdim], k + 1))
    want = O.sweep_collocated(st, ns, k, dim, tdim, sig, tier, ndouble)
    plan = sl.Plan(ns, k, tier, ndouble=ndouble)
    m_in, h_in = upload_nd(st, plan)
    m_out, h_out = plan.empty_state()
    plan.advect_dim_collocated(dim, tdim, _dev(sig), m_in, h_in, m_out, h_out)
    got = download_nd(m_out, h_out, plan)
    keep = O.fp64_modes(ndim, k, ndouble).astype(bool)
    scale = float(np.max(np.abs(want)))
    big = np.maximum(np.abs(got), np.abs(want))
    tol = np.where(keep[:, None], 0.0, ulp(big, tier)) + 1e-13 * scale
    err = np.abs(got - want)
    assert np.all(err <= tol), (int(np.sum(err > tol)), float(np.max(err - tol)))


def test_equal_node_shifts_match_the_plain_sweep_on_the_gpu(sl):
    ns, k = (32, 20), 2
    st = inputs.random_coefficients(2, k, ns[0] * ns[1], seed=5)
    line = np.random.default_rng(5).uniform(-3, 3, ns[1])
    plan = sl.Plan(ns, k, "fp64")
    a = upload(st, "fp64")
    b1, b2 = plan.empty_state(), plan.empty_state()
    plan.advect_dim_collocated(0, 1, _dev(np.repeat(line[:, None], k + 1, axis=1)), *a, *b1)
    plan.advect_dim(0, _dev(line), 2, *a, *b2)
    x, y = download(*b1), download(*b2)
    assert np.max(np.abs(x - y)) <= 1e-14 * np.max(np.abs(y))
    assert abs(math.fsum(x[0].tolist()) - math.fsum(st[0].tolist())) <= 1e-14 * np.sum(np.abs(st[0]))


def test_collocation_beats_cell_centres_on_a_shear_flow(sl):
    nx, nv, k, T, nsteps = 64, 16, 2, 1.0, 10
    L = 2 * math.pi
    los, his = (0.0, -3.0), (L, 3.0)
    st = O.project_separable([(np.sin, lambda v: np.exp(-v * v / 2))], (nx, nv), los, his, k, nq=8)
    hx, hv, dt = L / nx, 6.0 / nv, T / nsteps
    xi, _ = O.gauss_legendre(k + 1)
    vc = -3.0 + (np.arange(nv) + 0.5) * hv
    node = _dev((vc[:, None] + 0.5 * hv * xi[None, :]) * dt / hx)
    line = _dev(vc * dt / hx)
    plan = sl.Plan((nx, nv), k, "fp64")
    c = [upload(st, "fp64"), plan.empty_state()]
    p = [upload(st, "fp64"), plan.empty_state()]
    for n in range(nsteps):
        plan.advect_dim_collocated(0, 1, node, *c[n % 2], *c[1 - n % 2])
        plan.advect_dim(0, line, 2, *p[n % 2], *p[1 - n % 2])
    exact = [(np.sin, lambda v: np.cos(v * T) * np.exp(-v * v / 2)),
             (lambda x: -np.cos(x), lambda v: np.sin(v * T) * np.exp(-v * v / 2))]
    want = O.project_separable(exact, (nx, nv), los, his, k, nq=8)
    w = O.mode_weights(2, k)[:, None]
    rel = lambda a: math.sqrt(np.sum(w * (a - want) ** 2) / np.sum(w * want ** 2))
    e_col, e_cc = rel(download(*c[nsteps % 2])), rel(download(*p[nsteps % 2]))
    assert e_col < e_cc / 100, (e_col, e_cc)


def test_collocated_sweep_rejects_bad_arguments(sl):
    plan = sl.Plan((8, 6), 1, "fp64")
    m, h = plan.empty_state()
    m2, h2 = plan.empty_state()
    sig = _dev(np.zeros(16))
    with pytest.raises(sl.SldgError) as ei:
        plan.advect_dim_collocated(0, 0, sig, m, h, m2, h2)
    assert ei.value.status == sl.SLDG_ERR_ARG
    with pytest.raises(sl.SldgError) as ei:
        plan.advect_dim_collocated(0, 1, sig, m, h, m, h)
    assert ei.value.status == sl.SLDG_ERR_ALIAS
