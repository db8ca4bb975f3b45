"""Full-size parity on the benchmark's grid: the 4D workload at 48^4 cells,
k = 2, 81 coefficients per cell.

* Every sweep direction, in the FP64, FP32-mode, BF16-mode and FP16-mode
  tiers, under every launch shape the autotuner can choose (the shapes the
  benchmark may time).  Each sweep is compared with the oracle on sampled output cells, with
  the single-sweep element bound, and each shape must reproduce the first one
  bitwise (a shape splits the work differently, never the arithmetic).
* Every sweep direction with scaled FP16 storage under every launch shape:
  exponents and absmax exactly as the oracle's scaling policy decides them
  (they depend on the whole output), values on sampled cells within the FP16
  bound at each plane's scale, and every shape bitwise equal to the first.
* One whole split step (6 sweeps) in FP32-mode and BF16-mode against the
  oracle's FP64 step, in the weighted L2 norm, with the mass drift.

Inputs: the benchmark's seeded random coefficients (Vlasov magnitude profile)
and the workload's seeded fields.
"""
import math

import numpy as np
import pytest

from oracle import sldg_oracle as O
from paper_1603_07008_amd import inputs
from gpu_helpers import assert_sweep_close, have_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sl():
    if not have_gpu():
        pytest.skip("no HIP device")
    import paper_1603_07008_amd as sl
    sl.lib()
    return sl


@pytest.fixture(scope="module")
def big():
    prob = inputs.vlasov_4d(n=48)
    st = inputs.random_coefficients(prob.ndim, prob.k, prob.cells, seed=1603)
    return prob, st


def _sample(prob, n, seed):
    """Random output cells plus the cells at both ends of every dimension."""
    rng = np.random.default_rng(seed)
    cells = set(rng.choice(prob.cells, n, replace=False).tolist())
    ns = prob.ns
    for corner in range(1 << prob.ndim):
        idx, stride = 0, 1
        for e in range(prob.ndim):
            idx += (ns[e] - 1 if corner >> e & 1 else 0) * stride
            stride *= ns[e]
        cells.add(idx)
    return np.array(sorted(cells), dtype=np.int64)


def _upload(sl, torch, state, tier):
    mass = torch.from_numpy(np.ascontiguousarray(state[0])).cuda()
    h64 = torch.from_numpy(state[1:]).cuda()
    hi = h64.to(sl.hi_dtype(tier)).contiguous()
    assert torch.equal(hi.to(torch.float64), h64), "state not representable in the tier"
    del h64
    return mass, hi


def _gather(torch, mass, hi, sel_d):
    m = mass.index_select(0, sel_d).to(torch.float64)
    h = hi.index_select(1, sel_d).to(torch.float64)
    return torch.cat([m[None], h], 0).cpu().numpy()


@pytest.mark.parametrize("tier", ["fp32", "fp64", "bf16", "fp16"])
def test_full_size_sweeps_every_direction_and_launch_shape(sl, big, tier):
    import torch
    prob, st0 = big
    state = O.to_tier(st0, tier)
    plan = sl.Plan(prob.ns, prob.k, tier)
    m_in, h_in = _upload(sl, torch, state, tier)
    m_out, h_out = plan.empty_state()
    sel = _sample(prob, 3000, 7)
    sel_d = torch.from_numpy(sel).cuda()
    seen = set()
    for sw in prob.seq:
        if sw.dim in seen:
            continue
        seen.add(sw.dim)
        want = O.sweep(state, prob.ns, prob.k, sw.dim, sw.sigma, sw.dep, tier, sel=sel)
        mag = O.sweep(state, prob.ns, prob.k, sw.dim, sw.sigma, sw.dep, sel=sel, absolute=True)
        shift = torch.from_numpy(sw.sigma).cuda()
        first = None
        for shape in sl.tune_candidates(sw.dim > 0):
            plan.set_shape(sw.dim, shape["rows"], shape["tuples"], shape["colwaves"])
            plan.advect_dim(sw.dim, shift, sw.dep_mask, m_in, h_in, m_out, h_out)
            got = _gather(torch, m_out, h_out, sel_d)
            if first is None:
                assert_sweep_close(got, want, mag, tier, prob.k, f"{tier} dim {sw.dim} {shape}")
                first = got
            else:
                assert np.array_equal(got, first), f"{tier} dim {sw.dim}: shape {shape} differs"
    plan.close()


@pytest.mark.parametrize("tier", ["fp32", "bf16", "fp16"])
def test_full_size_staged_sweeps_are_bitwise_the_direct_sweeps(sl, big, tier):
    """The v sweeps of the 48^4 workload staged through LDS, on every cell:
    bitwise the direct strided kernel's results (section II-A update; the
    staged form changes only how the source values reach the threads)."""
    import torch
    prob, st0 = big
    state = O.to_tier(st0, tier)
    plan = sl.Plan(prob.ns, prob.k, tier)
    s_in = _upload(sl, torch, state, tier)
    ity = torch.int32 if tier == "fp32" else torch.int16
    for sw in prob.seq:
        if sw.dim < 2:
            continue
        shift = torch.from_numpy(sw.sigma).cuda()
        plan.set_shape(sw.dim, 4, 9, 2)
        ref = plan.empty_state()
        assert plan.sweep_form(sw.dim, sw.dep_mask, s_in, ref) == "strided"
        plan.advect_dim(sw.dim, shift, sw.dep_mask, *s_in, *ref)
        for rows, tuples, cw in ((4, 27, 2), (4, 27, 4), (8, 9, 2), (4, 9, 1)):
            plan.set_shape(sw.dim, rows, tuples, cw | sl.SLDG_SHAPE_STAGED)
            out = plan.empty_state()
            assert plan.sweep_form(sw.dim, sw.dep_mask, s_in, out) == "staged"
            plan.advect_dim(sw.dim, shift, sw.dep_mask, *s_in, *out)
            torch.cuda.synchronize()
            what = f"{tier} dim {sw.dim} rows {rows} tuples {tuples} cw {cw}"
            assert torch.equal(out[0], ref[0]), what
            assert torch.equal(out[1].view(ity), ref[1].view(ity)), what
            del out
        del ref
    plan.close()


@pytest.mark.parametrize("tier,tol", [("fp32", 1e-6), ("bf16", 5e-3)])
def test_full_size_split_step_against_fp64_oracle(sl, big, tier, tol):
    import torch
    prob, st0 = big
    seq_o = [(s.dim, s.sigma, s.dep) for s in prob.seq]
    ref = O.run_sequence(st0, prob.ns, prob.k, seq_o, "fp64", 1)
    state = O.to_tier(st0, tier)
    plan = sl.Plan(prob.ns, prob.k, tier)
    s0 = _upload(sl, torch, state, tier)
    s1 = plan.empty_state()
    seq = [(s.dim, s.dep_mask, torch.from_numpy(s.sigma).cuda()) for s in prob.seq]
    plan.tune(seq, s0, s1, reps=1)
    res = plan.split_steps(seq, 1, s0, s1)
    mass, hi = (s0, s1)[res]
    m = mass.cpu().numpy()
    w = O.mode_weights(prob.ndim, prob.k)
    num = w[0] * np.sum((m - ref[0]) ** 2)
    den = w[0] * np.sum(ref[0] ** 2)
    hcpu = hi.cpu()
    for p in range(prob.modes - 1):
        d = hcpu[p].to(torch.float64).numpy()
        num += w[p + 1] * np.sum((d - ref[p + 1]) ** 2)
        den += w[p + 1] * np.sum(ref[p + 1] ** 2)
    rel = math.sqrt(num / den)
    assert rel < tol, rel
    m0, m1 = O.mass_sum(state[0]), O.mass_sum(m)
    assert abs(m1 - m0) <= 1e-14 * abs(m0)
    plan.close()


@pytest.mark.parametrize("dim", [0, 1, 2, 3])
def test_full_size_scaled_fp16_sweep_every_launch_shape(sl, big, dim):
    import torch
    from test_gpu_scaled import _check_sweep
    prob, st0 = big
    sw = next(s for s in prob.seq if s.dim == dim)
    vals, e_in, a_in = O.to_scaled(st0, prob.k, prob.ndim)
    want = O.sweep_scaled(vals, e_in, a_in, prob.ns, prob.k, dim, sw.sigma, sw.dep)
    sel = _sample(prob, 3000, 11 + dim)
    mag = O.sweep(vals, prob.ns, prob.k, dim, sw.sigma, sw.dep, sel=sel, absolute=True)
    want_sel = (want[0][:, sel], want[1], want[2])
    plan = sl.Plan(prob.ns, prob.k, "fp16")
    # upload the scaled state: FP16 planes hold value * 2^e
    m_in = torch.from_numpy(np.ascontiguousarray(vals[0])).cuda()
    h_in = torch.empty((plan.n_hi, plan.cells), dtype=torch.float16, device="cuda")
    for p in range(plan.n_hi):
        row = torch.from_numpy(np.ldexp(vals[p + 1], int(e_in[p + 1]))).cuda()
        h_in[p] = row.to(torch.float16)
        assert torch.equal(h_in[p].to(torch.float64), row), "not an FP16 state"
    del vals, want
    s_in = plan.empty_scale()
    s_in[0] = torch.from_numpy(e_in[1:].astype(np.int32)).cuda()
    s_in[1] = torch.from_numpy(a_in[1:].astype(np.float32).view(np.int32)).cuda()
    m_out, h_out = plan.empty_state()
    s_out = plan.empty_scale()
    sel_d = torch.from_numpy(sel).cuda()
    shift = torch.from_numpy(sw.sigma).cuda()
    keep = O.fp64_modes(prob.ndim, prob.k).astype(bool)
    first = None
    for shape in sl.tune_candidates(dim > 0):
        plan.set_shape(dim, shape["rows"], shape["tuples"], shape["colwaves"])
        plan.advect_dim_scaled(dim, shift, sw.dep_mask, m_in, h_in, s_in, m_out, h_out, s_out)
        sc = s_out.cpu().numpy()
        e_h = sc[0].astype(np.int64)
        a_h = sc[1].view(np.float32).astype(np.float64)
        raw = _gather(torch, m_out, h_out, sel_d)
        if first is None:
            vals_g = raw.copy()
            vals_g[1:] = np.ldexp(raw[1:], -e_h[:, None])
            e = np.concatenate([[0], e_h])
            a = np.concatenate([[0.0], a_h])
            _check_sweep((vals_g, e, a), want_sel, mag, keep, prob.k, f"scaled dim {dim}")
            first = (raw, sc)
        else:
            assert np.array_equal(raw, first[0]) and np.array_equal(sc, first[1]), \
                f"scaled dim {dim}: shape {shape} differs"
    plan.close()


@pytest.mark.parametrize("tier", ["fp32", "bf16", "fp64", "fp16"])
def test_full_size_fused_step_is_bitwise_the_unfused_step(sl, big, tier):
    """One split step at 48^4 with the (x1, x2) pairs fused (the benchmark's
    step) and with every sweep its own pass: the same bits, with the fused
    pass really taken (two fused launches per step)."""
    import torch
    prob, st0 = big
    state = O.to_tier(st0, tier)
    plan = sl.Plan(prob.ns, prob.k, tier)
    seq = [(s.dim, s.dep_mask, torch.from_numpy(s.sigma).cuda()) for s in prob.seq]
    out = {}
    for fuse in (True, False):
        plan.set_fusion(fuse)
        s0 = _upload(sl, torch, state, tier)
        s1 = plan.empty_state()
        plan.timing_enable(True)
        res = plan.split_steps(seq, 1, s0, s1)
        n_fused, _ = plan.timing_read(-3)
        plan.timing_enable(False)
        assert n_fused == (2 if fuse else 0)
        out[fuse] = (s0, s1)[res]
        del s0, s1
    for a, b in zip(out[True], out[False]):
        assert torch.equal(a.view(torch.uint8), b.view(torch.uint8)), tier
    plan.close()


@pytest.mark.parametrize("tier", ["fp32", "bf16"])
def test_full_size_memory_order_covers_every_cell(sl, big, tier):
    """The v sweeps of the 48^4 workload with memory-order tiles
    (SLDG_SHAPE_MEMORDER; v1 in dispatch order, v2 in XCD runs), direct and
    staged: outputs filled with NaN beforehand, every cell bitwise the
    default order's result, so that no tile is skipped or written twice
    with other data (section II-A update; the order changes no arithmetic)."""
    import torch
    prob, st0 = big
    state = O.to_tier(st0, tier)
    plan = sl.Plan(prob.ns, prob.k, tier)
    s_in = _upload(sl, torch, state, tier)
    ity = torch.int32 if tier == "fp32" else torch.int16
    mo = sl.SLDG_SHAPE_MEMORDER
    for sw in prob.seq:
        if sw.dim < 2:
            continue
        shift = torch.from_numpy(sw.sigma).cuda()
        plan.set_shape(sw.dim, 8, 3, 4)
        ref = plan.empty_state()
        plan.advect_dim(sw.dim, shift, sw.dep_mask, *s_in, *ref)
        out = plan.empty_state()
        for rows, tuples, cw in ((8, 3, 4 | mo), (4, 9, 4 | mo), (8, 9, 2 | mo),
                                 (4, 27, 4 | mo | sl.SLDG_SHAPE_STAGED),
                                 (8, 9, 2 | mo | sl.SLDG_SHAPE_STAGED)):
            plan.set_shape(sw.dim, rows, tuples, cw)
            out[0].fill_(float("nan"))
            out[1].fill_(float("nan"))
            plan.advect_dim(sw.dim, shift, sw.dep_mask, *s_in, *out)
            torch.cuda.synchronize()
            what = f"{tier} dim {sw.dim} rows {rows} tuples {tuples} colwaves {cw}"
            assert torch.equal(out[0], ref[0]), what
            assert torch.equal(out[1].view(ity), ref[1].view(ity)), what
    plan.close()
