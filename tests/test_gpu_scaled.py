"""GPU parity of FP16 storage with per-plane power-of-two scaling (the
sldg_scaled_* and sldg_*_scaled entry points) against the oracle's emulation
(oracle.sldg_oracle.to_scaled / sweep_scaled), on the same seeded inputs.

* Import from FP64 is bit-exact: both sides take the exact absmax, the same
  exponent rule and a correctly rounded FP16 conversion.
* Export is exact.
* For a sweep, the exponents match exactly.  The stored values are compared
  element by element with the bound of the unscaled FP16 tier, taken at the
  plane's scale: the FP16 quantum of the plane, plus the FP32 accumulation
  error relative to sum |A x| + |B y|.  Every covered case has the absmax of
  each plane away from a binade edge by far more than the FP32 error, so the
  exponent decisions agree.
"""
import math
import zlib

import numpy as np
import pytest

from oracle import sldg_oracle as O
from paper_1603_07008_amd import inputs
from gpu_helpers import gamma, have_gpu

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


def _split(plan):
    pm = plan.plane_map()
    lo = [m for _, m in sorted((-1 - v, m) for m, v in enumerate(pm) if v < 0)]
    hi = [m for _, m in sorted((v, m) for m, v in enumerate(pm) if v >= 0)]
    return lo, hi


def upload_scaled(plan, scaled):
    """Oracle (values, exps, amax) -> (mass, hi, scale) device tensors."""
    import torch
    vals, e, a = scaled
    lo, hi = _split(plan)
    mass = _dev(vals[lo].reshape(-1) if len(lo) == 1 else vals[lo])
    eh = np.array([e[m] for m in hi], dtype=np.int64)
    stored = np.ldexp(vals[hi], eh[:, None])
    h = torch.from_numpy(stored.reshape(len(hi), vals.shape[1])).to(torch.float16)
    assert torch.equal(h.to(torch.float64), torch.from_numpy(stored)), "not an FP16 state"
    scale = torch.empty((2, len(hi)), dtype=torch.int32)
    scale[0] = torch.from_numpy(eh.astype(np.int32))
    scale[1] = torch.from_numpy(np.array([a[m] for m in hi], dtype=np.float32).view(np.int32))
    return mass.contiguous(), h.cuda().contiguous(), scale.cuda().contiguous()


def download_scaled(plan, mass, hi, scale):
    """Device state -> (values, exps, amax) in the oracle's mode-major form."""
    import torch
    lo, hi_modes = _split(plan)
    m = mass.detach().cpu().to(torch.float64).numpy().reshape(len(lo), plan.cells)
    sc = scale.detach().cpu().numpy()
    e_h = sc[0].astype(np.int64)
    a_h = sc[1].view(np.float32).astype(np.float64)
    h = hi.detach().cpu().to(torch.float64).numpy().reshape(len(hi_modes), plan.cells)
    vals = np.empty((plan.modes, plan.cells))
    e = np.zeros(plan.modes, dtype=np.int64)
    a = np.zeros(plan.modes)
    for i, mode in enumerate(lo):
        vals[mode] = m[i]
    for i, mode in enumerate(hi_modes):
        vals[mode] = np.ldexp(h[i], -e_h[i])
        e[mode], a[mode] = e_h[i], a_h[i]
    return vals, e, a


def _vlasov_state(nx, nv, unit=1.0):
    prob = inputs.vlasov_2d(nx=nx, nv=nv)
    st = O.project_separable(prob.f0_terms, prob.ns, prob.los, prob.his, prob.k)
    return prob, st * unit


def _random_state(ns, k, seed):
    rng = np.random.default_rng(seed)
    ndim = len(ns)
    st = inputs.random_coefficients(ndim, k, int(np.prod(ns)), seed=seed)
    return st * (1.0 + 0.01 * rng.standard_normal(st.shape[0]))[:, None]


def _check_sweep(got, want, mag, keep, k, what):
    """Element-wise bound at the scale of each plane."""
    gv, ge, ga = got
    wv, we, wa = want
    narrow = ~keep
    assert np.array_equal(ge[narrow], we[narrow]), f"{what}: exponents {ge} vs {we}"
    np.testing.assert_allclose(ga[narrow], wa[narrow], rtol=2.0 ** -20, atol=0, err_msg=what)
    big = np.maximum(np.abs(gv), np.abs(wv))
    for m in range(gv.shape[0]):
        if keep[m]:
            tol = np.spacing(big[m]) + gamma("fp64", k, True) * mag[m]
        else:
            s = np.ldexp(big[m], int(we[m]))                 # stored magnitude
            ex = np.floor(np.log2(np.where(s > 0, s, 1.0)))
            q = np.ldexp(1.0, (np.maximum(ex, -14) - 10).astype(int))
            tol = np.ldexp(q, -int(we[m])) + gamma("fp16", k, False) * mag[m]
        err = np.abs(gv[m] - wv[m])
        assert np.all(err <= tol), (f"{what}: mode {m}: {int(np.sum(err > tol))} elements out "
                                    f"of bound, worst {np.max(err - tol):.3g}")


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("unit", [1.0, 2.0 ** -40, 1e6])
def test_import_is_bit_exact_and_export_exact(sl, unit):
    import torch
    prob, st = _vlasov_state(64, 48, unit)
    st[5] = 0.0                                              # an all-zero plane
    plan = sl.Plan(prob.ns, prob.k, "fp16")
    want = O.to_scaled(st, prob.k, prob.ndim)
    hi = torch.empty((plan.n_hi, plan.cells), dtype=torch.float16, device="cuda")
    scale = plan.empty_scale()
    plan.scaled_import(_dev(st[1:]), hi, scale)
    got = download_scaled(plan, _dev(st[0]), hi, scale)
    assert np.array_equal(got[1], want[1])
    assert np.array_equal(got[2], want[2])
    assert np.array_equal(got[0], want[0])
    back = plan.scaled_export(hi, scale).cpu().numpy()
    assert np.array_equal(back, want[0][1:])


CASES = [
    # ns, k, dim, dep, seed
    ((48, 40), 2, 0, (1,), 1),          # dimension-0 window form
    ((48, 40), 2, 1, (0,), 2),          # strided, per-lane shifts
    ((45, 16), 2, 0, (1,), 3),          # dimension-0 generic form (N_0 odd)
    ((12, 10, 9), 1, 2, (0, 1), 4),     # strided, partial row chunk, ragged columns
    ((12, 10, 9), 3, 1, (2,), 5),
    ((16, 6, 5), 3, 0, (2,), 6),
    # 4D (x1, x2, v1, v2): every sweep direction of the split step
    ((10, 8, 6, 5), 2, 0, (2,), 10),    # dimension-0 window form, shift from v1
    ((10, 8, 6, 5), 2, 1, (3,), 11),    # strided x2, shift from v2
    ((10, 8, 6, 5), 2, 2, (0, 1), 12),  # strided v1, per-lane shifts from (x1, x2)
    ((9, 7, 5, 6), 1, 3, (0, 1), 13),   # strided v2, ragged columns
    ((9, 7, 5, 6), 3, 0, (2,), 14),     # dimension-0 generic form (N_0 odd)
]


@pytest.mark.parametrize("ns,k,dim,dep,seed", CASES)
def test_scaled_sweep_matches_oracle(sl, ns, k, dim, dep, seed):
    st = _random_state(ns, k, seed)
    ndim = len(ns)
    plan = sl.Plan(ns, k, "fp16")
    rng = np.random.default_rng(100 + seed)
    ntab = int(np.prod([ns[e] for e in dep])) if dep else 1
    sigma = rng.uniform(-3.0, 3.0, ntab)
    scaled = O.to_scaled(st, k, ndim)
    want = O.sweep_scaled(*scaled, ns, k, dim, sigma, dep)
    mag = O.sweep(scaled[0], ns, k, dim, sigma, dep, absolute=True)
    m_in, h_in, s_in = upload_scaled(plan, scaled)
    m_out, h_out = plan.empty_state()
    s_out = plan.empty_scale()
    mask = sum(1 << e for e in dep)
    plan.advect_dim_scaled(dim, _dev(sigma), mask, m_in, h_in, s_in, m_out, h_out, s_out)
    got = download_scaled(plan, m_out, h_out, s_out)
    _check_sweep(got, want, mag, O.fp64_modes(ndim, k).astype(bool), k, f"{ns} dim {dim}")


def test_scaled_sweep_repairs_a_plane_that_outgrows_its_headroom(sl):
    n0, n1, k = 64, 8, 2
    rng = np.random.default_rng(7)
    st = np.zeros(((k + 1) ** 2, n0 * n1))
    cells = np.arange(n0 * n1)
    st[0] = np.where(cells % n0 < n0 // 2, 1.0, 0.25)        # a step along dimension 0
    st[1:] = 1e-12 * rng.standard_normal((st.shape[0] - 1, st.shape[1]))
    scaled = O.to_scaled(st, k, 2)
    sigma = np.full(n1, 0.3)
    want = O.sweep_scaled(*scaled, (n0, n1), k, 0, sigma, (1,))
    repaired = [m for m in range(1, st.shape[0])
                if math.ldexp(want[2][m], O.storage_exponent(scaled[2][m], O.SCALE_HEADROOM))
                >= 2.0 ** 15]
    assert repaired, "the case must exercise the repair"
    mag = O.sweep(scaled[0], (n0, n1), k, 0, sigma, (1,), absolute=True)
    plan = sl.Plan((n0, n1), k, "fp16")
    m_in, h_in, s_in = upload_scaled(plan, scaled)
    m_out, h_out = plan.empty_state()
    s_out = plan.empty_scale()
    plan.advect_dim_scaled(0, _dev(sigma), 2, m_in, h_in, s_in, m_out, h_out, s_out)
    got = download_scaled(plan, m_out, h_out, s_out)
    assert np.all(np.isfinite(got[0]))
    _check_sweep(got, want, mag, O.fp64_modes(2, k).astype(bool), k, "repair")


def test_scaled_sweeps_are_invariant_under_powers_of_two(sl):
    import torch
    prob, st = _vlasov_state(64, 48)
    plan = sl.Plan(prob.ns, prob.k, "fp16")
    seq = [(s.dim, s.dep_mask, _dev(s.sigma)) for s in prob.seq]
    outs = []
    for t in (0, -40):
        m0, h0, s0 = upload_scaled(plan, O.to_scaled(np.ldexp(st, t), prob.k, prob.ndim))
        m1, h1 = plan.empty_state()
        s1 = plan.empty_scale()
        res = plan.split_steps_scaled(seq, 3, (m0, h0, s0), (m1, h1, s1))
        bufs = [(m0, h0, s0), (m1, h1, s1)]
        outs.append(download_scaled(plan, *bufs[res]))
    torch.cuda.synchronize()
    assert np.array_equal(outs[1][0], np.ldexp(outs[0][0], -40))
    assert np.array_equal(outs[1][1][1:], outs[0][1][1:] + 40)


def test_scaled_split_steps_match_single_sweeps_and_oracle(sl):
    import torch
    prob, st = _vlasov_state(64, 48)
    steps = 10
    seq_o = [(s.dim, s.sigma, s.dep) for s in prob.seq]
    plan = sl.Plan(prob.ns, prob.k, "fp16")
    seq = [(s.dim, s.dep_mask, _dev(s.sigma)) for s in prob.seq]
    scaled = O.to_scaled(st, prob.k, prob.ndim)
    # split steps
    a0 = upload_scaled(plan, scaled)
    a1 = (*plan.empty_state(), plan.empty_scale())
    res = plan.split_steps_scaled(seq, steps, a0, a1)
    got = download_scaled(plan, *(a0, a1)[res])
    # the same sweeps one by one
    cur = upload_scaled(plan, scaled)
    nxt = (*plan.empty_state(), plan.empty_scale())
    for _ in range(steps):
        for dim, mask, sh in seq:
            plan.advect_dim_scaled(dim, sh, mask, *cur, *nxt)
            cur, nxt = nxt, cur
    one = download_scaled(plan, *cur)
    torch.cuda.synchronize()
    for x, y in zip(got, one):
        assert np.array_equal(x, y)
    # against the oracle's scaled run and the FP64 run
    want = O.run_sequence_scaled(scaled, prob.ns, prob.k, seq_o, steps)
    ref = O.run_sequence(st, prob.ns, prob.k, seq_o, "fp64", steps)
    w = O.mode_weights(prob.ndim, prob.k)[:, None]
    rel = lambda a, b: math.sqrt(np.sum(w * (a - b) ** 2) / np.sum(w * b ** 2))
    assert rel(got[0], want[0]) < 1e-3
    assert rel(got[0], ref) < 5e-3
    m0 = O.mass_sum(st[0])
    assert abs(O.mass_sum(got[0][0]) - m0) <= 1e-14 * abs(m0)


def test_scaled_sweep_with_leading_fp64_modes(sl):
    ns, k, ndouble = (32, 24), 2, 2
    st = _random_state(ns, k, 9)
    plan = sl.Plan(ns, k, "fp16", ndouble=ndouble)
    scaled = O.to_scaled(st, k, 2, ndouble=ndouble)
    sigma = np.random.default_rng(9).uniform(-2, 2, ns[0])
    want = O.sweep_scaled(*scaled, ns, k, 1, sigma, (0,), ndouble=ndouble)
    mag = O.sweep(scaled[0], ns, k, 1, sigma, (0,), absolute=True)
    m_in, h_in, s_in = upload_scaled(plan, scaled)
    m_out, h_out = plan.empty_state()
    s_out = plan.empty_scale()
    plan.advect_dim_scaled(1, _dev(sigma), 1, m_in, h_in, s_in, m_out, h_out, s_out)
    got = download_scaled(plan, m_out, h_out, s_out)
    _check_sweep(got, want, mag, O.fp64_modes(2, k, ndouble).astype(bool), k, "ndouble=2")


def test_scaled_entry_points_reject_bad_arguments(sl):
    import torch
    p32 = sl.Plan((16, 8), 1, "fp32")
    m, h = p32.empty_state()
    sc = torch.zeros((2, p32.n_hi), dtype=torch.int32, device="cuda")
    with pytest.raises(sl.SldgError) as ei:
        p32.advect_dim_scaled(0, _dev([0.1]), 0, m, h, sc, *p32.empty_state(), sc.clone())
    assert ei.value.status == sl.SLDG_ERR_UNSUPPORTED
    p16 = sl.Plan((16, 8), 1, "fp16")
    m0, h0 = p16.empty_state()
    m1, h1 = p16.empty_state()
    s0 = torch.zeros((2, p16.n_hi), dtype=torch.int32, device="cuda")
    with pytest.raises(sl.SldgError) as ei:
        p16.advect_dim_scaled(0, _dev([0.1]), 0, m0, h0, s0, m1, h1, s0)
    assert ei.value.status == sl.SLDG_ERR_ALIAS
    with pytest.raises(sl.SldgError) as ei:
        p16.set_scale_headroom(15)
    assert ei.value.status == sl.SLDG_ERR_ARG


TWO_SHIFT_SCALED = [
    # ns, k, swept dim, dep: partial waves, row counts that 8 does not divide
    ((37, 19), 3, 1, (0,)),
    ((96, 13, 3), 2, 1, (0,)),
    ((48, 4, 9, 10), 2, 3, (0, 1)),
]


@pytest.mark.parametrize("field", ["zero", "int"])
@pytest.mark.parametrize("ns,k,dim,dep", TWO_SHIFT_SCALED)
def test_scaled_two_shift_waves_agree_across_shapes(sl, ns, k, dim, dep, field):
    """Scaled FP16 sweeps whose waves hold two neighbouring integer shifts
    (s = N-1 next to 0, or 2 next to 3): every strided launch shape, with
    tiles in either order, gives the lane form's values, exponents and
    absmax bits (the per-wave absmax partials see the same outputs), and the
    result stays within the oracle's bound (section II-A update)."""
    import torch
    ndim = len(ns)
    st = _random_state(ns, k, 77)
    plan = sl.Plan(ns, k, "fp16")
    rng = np.random.default_rng(zlib.crc32(repr((ns, k, dim, field)).encode()))
    ntab = int(np.prod([ns[e] for e in dep]))
    sigma = rng.uniform(-0.01, 0.01, ntab) + (3.0 if field == "int" else 0.0)
    scaled = O.to_scaled(st, k, ndim)
    m_in, h_in, s_in = upload_scaled(plan, scaled)
    mask = sum(1 << e for e in dep)
    ref = None
    shapes = ((0, 0, 1), (1, 1, 1), (4, 1, 2), (8, 0, 1), (8, 3, 4),
              (8, 3, 4 | sl.SLDG_SHAPE_MEMORDER), (4, 1, 1 | sl.SLDG_SHAPE_MEMORDER))
    for rows, tuples, cw in shapes:
        plan.set_shape(dim, rows, tuples, cw)
        m_out, h_out = plan.empty_state()
        s_out = plan.empty_scale()
        plan.advect_dim_scaled(dim, _dev(sigma), mask, m_in, h_in, s_in, m_out, h_out, s_out)
        torch.cuda.synchronize()
        got = (m_out.cpu(), h_out.cpu().view(torch.int16), s_out.cpu())
        if ref is None:
            ref = got
            want = O.sweep_scaled(*scaled, ns, k, dim, sigma, dep)
            mag = O.sweep(scaled[0], ns, k, dim, sigma, dep, absolute=True)
            _check_sweep(download_scaled(plan, m_out, h_out, s_out), want, mag,
                         O.fp64_modes(ndim, k).astype(bool), k, f"{ns} dim {dim} {field}")
        else:
            for a, b, nm in zip(got, ref, ("mass", "hi", "scale")):
                assert torch.equal(a, b), (rows, tuples, cw, nm)
    plan.close()
