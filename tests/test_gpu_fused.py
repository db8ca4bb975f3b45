"""The fused pair of sweeps along dimensions 0 and 1 (sldg_advect_dims01):
one pass over the state that applies the dimension-0 sweep and then the
dimension-1 sweep of a split step (section II; each sweep the update rule of
section II-A).  It must give bitwise the result of the two sweeps run one
after the other (the intermediate state rounded to the storage tier as the
unfused path stores it), in every tier and degree, for tiles that cover a
slab's rows with a ragged last chunk, for displacements of both signs and
larger than the grid, and split steps must give the same bits with fusion on
and off.  A direct check against the FP64 oracle's two sweeps is included."""
import math

import numpy as np
import pytest

from oracle import sldg_oracle as O
from paper_1603_07008_amd import inputs
from gpu_helpers import download, have_gpu, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sl():
    if not have_gpu():
        pytest.skip("no HIP device")
    import paper_1603_07008_amd as sl
    sl.lib()
    return sl


def _state(sl, plan, seed):
    m, h = inputs.random_coefficients_device(len(plan.ncells), plan.k, plan.cells, seed=seed)
    return m.contiguous(), h.to(sl.hi_dtype(plan.tier)).contiguous()


def _shift(ns, dep, seed, spread):
    import torch
    n = 1
    for e in dep:
        n *= ns[e]
    return torch.from_numpy(np.random.default_rng(seed).uniform(-spread, spread, n)).cuda()


def _mask(dep):
    return sum(1 << e for e in dep)


def _bits(t):
    import torch
    return t.view(torch.uint8)


def _unfused(plan, s0, d0, s1, d1, state):
    tmp = plan.empty_state()
    out = plan.empty_state()
    plan.advect_dim(0, s0, _mask(d0), *state, *tmp)
    plan.advect_dim(1, s1, _mask(d1), *tmp, *out)
    return out


CASES = [
    # grid, dep of the dim-0 displacement, dep of the dim-1 displacement, spread (cells)
    ((48, 48, 6, 5), (2,), (3,), 1.3),
    ((48, 13, 7), (2,), (2,), 2.5),          # 13 rows: a ragged last row chunk
    ((12, 5, 3, 4), (2, 3), (3,), 40.0),     # displacements beyond the grid
    ((36, 1, 9), (2,), (2,), 3.0),           # one row along dimension 1
    ((64, 20), (), (), 0.37),                # a single slab, constant displacements
]


@pytest.mark.parametrize("tier", ["fp64", "fp32", "bf16", "fp16"])
@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_fused_pair_is_bitwise_two_sweeps(sl, tier, k, case):
    import torch
    ns, d0, d1, spread = CASES[case]
    plan = sl.Plan(ns, k, tier)
    s0 = _shift(ns, d0, 10 + case, spread)
    s1 = _shift(ns, d1, 20 + case, spread)
    st = _state(sl, plan, 30 + case)
    want = _unfused(plan, s0, d0, s1, d1, st)
    got = plan.empty_state()
    plan.advect_dims01(s0, _mask(d0), s1, _mask(d1), *st, *got)
    torch.cuda.synchronize()
    for a, b in zip(got, want):
        assert torch.equal(_bits(a), _bits(b)), f"{tier} k={k} {ns}"
    plan.close()


@pytest.mark.parametrize("rows", [1, 2, 3, 8, 16])
def test_every_tile_height_gives_the_same_bits(sl, rows, monkeypatch):
    import torch
    monkeypatch.setenv("SLDG_XY_ROWS", str(rows))
    ns = (48, 37, 4, 3)
    plan = sl.Plan(ns, 2, "fp32")            # reads the tile height when made
    s0 = _shift(ns, (2,), 1, 1.2)
    s1 = _shift(ns, (3,), 2, 1.2)
    st = _state(sl, plan, 3)
    want = _unfused(plan, s0, (2,), s1, (3,), st)
    got = plan.empty_state()
    plan.advect_dims01(s0, 4, s1, 8, *st, *got)
    torch.cuda.synchronize()
    for a, b in zip(got, want):
        assert torch.equal(_bits(a), _bits(b))
    plan.close()


@pytest.mark.parametrize("tier", ["fp64", "fp32"])
def test_fused_pair_matches_the_fp64_oracle(sl, tier):
    ns, k = (16, 12, 5), 2
    rng = np.random.default_rng(5)
    sig0 = rng.uniform(-1.5, 1.5, ns[2])
    sig1 = rng.uniform(-1.5, 1.5, ns[2])
    st = O.to_tier(inputs.random_coefficients(3, k, int(np.prod(ns)), seed=6), tier)
    plan = sl.Plan(ns, k, tier)
    import torch
    m, h = upload(st, tier)
    out = plan.empty_state()
    plan.advect_dims01(torch.from_numpy(sig0).cuda(), 4, torch.from_numpy(sig1).cuda(), 4, m, h,
                       *out)
    got = download(*out)
    mid = O.sweep(st, ns, k, 0, sig0, (2,), "fp64")
    want = O.sweep(mid, ns, k, 1, sig1, (2,), "fp64")
    w = O.mode_weights(3, k)[:, None]
    rel = math.sqrt(float(np.sum(w * (got - want) ** 2)) / float(np.sum(w * want ** 2)))
    assert rel <= (1e-13 if tier == "fp64" else 1e-6), rel
    if tier == "fp64":
        assert np.max(np.abs(got[0] - want[0])) <= 1e-14 * np.max(np.abs(want[0]))
    # the FP64 mass mode conserves the total mass in every tier (section II-A)
    m_in, m_out = math.fsum(st[0]), math.fsum(got[0])
    assert abs(m_out - m_in) <= 1e-14 * math.fsum(np.abs(st[0]))
    plan.close()


def test_split_steps_fuse_the_pair_and_keep_the_bits(sl):
    import torch
    prob = inputs.vlasov_4d(n=12)
    for tier in ("fp32", "bf16"):
        plan = sl.Plan(prob.ns, prob.k, tier)
        seq = [(sw.dim, sw.dep_mask, torch.from_numpy(sw.sigma).cuda()) for sw in prob.seq]
        st = _state(sl, plan, 7)
        res = {}
        for fuse in (False, True):
            plan.set_fusion(fuse)
            a = (st[0].clone(), st[1].clone())
            b = plan.empty_state()
            plan.timing_enable(True)
            r = plan.split_steps(seq, 3, a, b)
            n_fused, _ = plan.timing_read(-3)
            plan.timing_enable(False)
            res[fuse] = (a, b)[r]
            assert n_fused == (6 if fuse else 0)      # two (x1, x2) pairs per step
        for x, y in zip(res[False], res[True]):
            assert torch.equal(_bits(x), _bits(y)), tier
        plan.close()


def test_ineligible_pairs_are_refused_and_split_steps_fall_back(sl):
    import torch
    ns = (48, 8, 5)
    plan = sl.Plan(ns, 2, "fp32")
    st = _state(sl, plan, 8)
    out = plan.empty_state()
    s_v = _shift(ns, (2,), 9, 1.0)
    s_x = _shift(ns, (0,), 10, 1.0)
    with pytest.raises(sl.SldgError) as ei:
        plan.advect_dims01(s_v, 4, s_x, 1, *st, *out)     # dim-1 shift depends on dim 0
    assert ei.value.status == sl.SLDG_ERR_UNSUPPORTED
    p2 = sl.Plan((46, 8, 5), 2, "fp32")                    # rows not whole 4-cell blocks
    st2 = _state(sl, p2, 11)
    with pytest.raises(sl.SldgError) as ei:
        p2.advect_dims01(s_v, 4, s_v, 4, *st2, *p2.empty_state())
    assert ei.value.status == sl.SLDG_ERR_UNSUPPORTED
    p3 = sl.Plan(ns, 2, "fp32", ndouble=2)                 # more FP64 modes than the mean
    st3 = plan_state_nd(sl, p3)
    with pytest.raises(sl.SldgError) as ei:
        p3.advect_dims01(s_v, 4, s_v, 4, *st3, *p3.empty_state())
    assert ei.value.status == sl.SLDG_ERR_UNSUPPORTED
    # split steps with such a pair run every sweep unfused: same bits either way
    seq = [(0, 4, s_v), (1, 1, s_x)]
    outs = []
    for fuse in (False, True):
        plan.set_fusion(fuse)
        a = (st[0].clone(), st[1].clone())
        b = plan.empty_state()
        r = plan.split_steps(seq, 2, a, b)
        outs.append((a, b)[r])
    for x, y in zip(*outs):
        assert torch.equal(_bits(x), _bits(y))
    for p in (plan, p2, p3):
        p.close()


def plan_state_nd(sl, plan):
    import torch
    m, h = inputs.random_coefficients_device(len(plan.ncells), plan.k, plan.cells, seed=12)
    full = torch.cat([m[None], h], 0)
    pm = plan.plane_map()
    lo = [mm for _, mm in sorted((-1 - v, mm) for mm, v in enumerate(pm) if v < 0)]
    hi = [mm for _, mm in sorted((v, mm) for mm, v in enumerate(pm) if v >= 0)]
    return full[lo].contiguous(), full[hi].to(sl.hi_dtype(plan.tier)).contiguous()
