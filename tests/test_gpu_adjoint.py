"""GPU adjoint sweep and differentiation through split steps, against the
oracle's transpose and central finite differences."""
import math

import numpy as np
import pytest

from oracle import sldg_oracle as O
from paper_1603_07008_amd import inputs
from gpu_helpers import assert_sweep_close, download, have_gpu, upload, weighted_rel_l2

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


CASES = [((64,), 2, {0: ()}), ((37, 19), 3, {0: (1,), 1: (0,)}),
         ((48, 10), 2, {0: (1,), 1: (0,)}), ((12, 10, 8, 9), 2, {0: (2,), 1: (3,), 2: (0, 1), 3: (0, 1)}),
         ((6, 4, 5, 3), 1, {0: (2, 3), 1: (), 2: (0, 1, 3), 3: (1,)})]


@pytest.mark.parametrize("case", CASES, ids=["x".join(map(str, c[0])) + f"-k{c[1]}" for c in CASES])
def test_adjoint_sweep_matches_oracle_transpose(sl, case):
    import torch
    ns, k, deps = case
    cells = int(np.prod(ns))
    rng = np.random.default_rng(cells + k)
    g = rng.standard_normal(((k + 1) ** len(ns), cells))
    p = sl.Plan(ns, k, "fp64")
    gi = upload(g, "fp64")
    go = p.empty_state()
    for dim, dep in deps.items():
        nsig = int(np.prod([ns[e] for e in dep])) if dep else 1
        sig = rng.uniform(-2.5 * ns[dim], 2.5 * ns[dim], nsig)
        p.advect_dim_adjoint(dim, _dev(sig), sum(1 << e for e in dep), gi[0], gi[1], go[0], go[1])
        torch.cuda.synchronize()
        got = download(*go)
        want = O.sweep_adjoint(g, ns, k, dim, sig, dep)
        scale = np.max(np.abs(want)) + 1e-300
        assert np.max(np.abs(got - want)) <= 64 * np.finfo(float).eps * scale * (k + 1), (dim, np.max(np.abs(got - want)))
        # dot-product identity on the device results: <M x, y> = <x, M^T y>
        x = rng.standard_normal(g.shape)
        xi = upload(x, "fp64")
        mx = p.empty_state()
        p.advect_dim(dim, _dev(sig), sum(1 << e for e in dep), xi[0], xi[1], mx[0], mx[1])
        torch.cuda.synchronize()
        lhs = math.fsum((download(*mx) * g).ravel().tolist())
        rhs = math.fsum((x * got).ravel().tolist())
        assert abs(lhs - rhs) <= 1e-12 * math.sqrt(g.size) * (1 + abs(lhs))


NARROW = [((64,), 2, {0: ()}), ((37, 19), 3, {0: (1,), 1: (0,)}),
          ((48, 10), 2, {0: (1,), 1: (0,)}), ((12, 10, 8, 9), 2, {0: (2,), 1: (3,), 2: (0, 1)}),
          ((6, 4, 5, 3), 1, {0: (2, 3), 3: (1,)})]


@pytest.mark.parametrize("tier", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("case", NARROW, ids=["x".join(map(str, c[0])) + f"-k{c[1]}" for c in NARROW])
def test_adjoint_sweep_narrow_tiers_match_oracle(sl, case, tier):
    # The transpose sweep in a narrow tier is the forward kernels on the
    # transposed tables, so it rounds as a forward sweep does: each output is
    # the exact transpose sum up to the tier's accumulation error, rounded to
    # the storage type (mode 0 computed and stored in FP64).  Compared element
    # by element with the oracle's FP64 transpose rounded to the tier, under
    # the single-sweep bound with the transpose's own magnitude sums.
    import torch
    ns, k, deps = case
    cells = int(np.prod(ns))
    rng = np.random.default_rng(3 * cells + k)
    g = O.to_tier(inputs.random_coefficients(len(ns), k, cells, seed=cells + k), tier)
    p = sl.Plan(ns, k, tier)
    gi = upload(g, tier)
    go = p.empty_state()
    for dim, dep in deps.items():
        nsig = int(np.prod([ns[e] for e in dep])) if dep else 1
        sig = rng.uniform(-2.5 * ns[dim], 2.5 * ns[dim], nsig)
        p.advect_dim_adjoint(dim, _dev(sig), sum(1 << e for e in dep), gi[0], gi[1], go[0], go[1])
        torch.cuda.synchronize()
        got = download(*go)
        want = O.to_tier(O.sweep_adjoint(g, ns, k, dim, sig, dep), tier)
        mag = O.sweep_adjoint(g, ns, k, dim, sig, dep, absolute=True)
        assert_sweep_close(got, want, mag, tier, k, f"{tier} adjoint {ns} dim {dim}")
        # the mass output is a transpose sum in FP64 from exactly widened inputs
        m_ex = O.sweep_adjoint(g, ns, k, dim, sig, dep)[0]
        assert np.all(np.abs(got[0] - m_ex) <= 8 * (k + 1) * 2.0 ** -52 * mag[0] + 1e-300)
    p.close()


def _setup_diff(sl, n, steps):
    import torch
    prob = inputs.vlasov_2d_differentiation(n=n, steps=steps)
    c0 = O.project_separable(prob.f0_terms, prob.ns, prob.los, prob.his, prob.k)
    tgt = O.project_separable(prob.target_terms, prob.ns, prob.los, prob.his, prob.k) + prob.target_noise
    p = sl.Plan(prob.ns, prob.k, "fp64")
    seq = [(sw.dim, sw.dep_mask, _dev(sw.sigma)) for sw in prob.seq]
    vol = O.cell_volume(prob.ns, prob.los, prob.his)
    return prob, c0, tgt, p, seq, vol


def _loss_and_grad(sl, p, seq, steps, c0, tgt, vol, ckpt=None):
    import torch
    from paper_1603_07008_amd import autograd as AG
    m0, h0 = upload(c0, "fp64")
    m0.requires_grad_(True)
    h0.requires_grad_(True)
    tm, th = upload(tgt, "fp64")
    m1, h1 = AG.split_steps(p, seq, steps, m0, h0, checkpoint_every=ckpt)
    L = AG.weighted_l2_misfit(m1, h1, tm, th, 2, p.k, vol)
    L.backward()
    return float(L), np.concatenate([m0.grad.cpu().numpy()[None], h0.grad.cpu().numpy()])


def _loss_only(sl, p, seq, steps, c, tgt, vol):
    import torch
    from paper_1603_07008_amd import autograd as AG
    m0, h0 = upload(c, "fp64")
    tm, th = upload(tgt, "fp64")
    with torch.no_grad():
        m1, h1 = AG.split_steps(p, seq, steps, m0, h0)
        return float(AG.weighted_l2_misfit(m1, h1, tm, th, 2, p.k, vol))


def test_gradient_matches_oracle_adjoint_and_checkpointing_is_bitwise(sl):
    prob, c0, tgt, p, seq, vol = _setup_diff(sl, 64, 12)
    L, g = _loss_and_grad(sl, p, seq, prob.steps, c0, tgt, vol)
    _, g_ck = _loss_and_grad(sl, p, seq, prob.steps, c0, tgt, vol, ckpt=5)
    assert np.array_equal(g, g_ck)
    oseq = [(s.dim, s.sigma, s.dep) for s in prob.seq]
    cT = O.run_sequence(c0, prob.ns, prob.k, oseq, "fp64", prob.steps)
    w = O.mode_weights(2, prob.k)[:, None]
    gT = vol * w * (cT - tgt)
    g_or = O.run_sequence_adjoint(gT, prob.ns, prob.k, oseq, prob.steps)
    assert weighted_rel_l2(g, g_or, 2, prob.k) <= 1e-12
    L_or = 0.5 * vol * math.fsum((w * (cT - tgt) ** 2).ravel().tolist())
    assert abs(L - L_or) <= 1e-12 * L_or


@pytest.mark.parametrize("n,steps,ndir", [(64, 12, 8), (512, 50, 64)])
def test_gradient_matches_central_finite_differences(sl, n, steps, ndir):
    prob, c0, tgt, p, seq, vol = _setup_diff(sl, n, steps)
    L, g = _loss_and_grad(sl, p, seq, steps, c0, tgt, vol, ckpt=10)
    dirs = inputs.fd_directions(ndir, prob.modes, prob.cells)
    h = 1e-6
    eps = np.finfo(float).eps
    # the loss is quadratic in c0, so central differences are exact up to the
    # rounding of the two loss values.  Each value carries the rounding of the
    # forward run, |dc_T| <~ n_sweeps * eps * |c_T|, which enters the misfit
    # through (c_T - t): |dL| <~ n_sweeps * eps * vol * sum_m w_m |c_T - t| |c_T|
    m0, h0 = upload(c0, "fp64")
    from paper_1603_07008_amd import autograd as AG
    import torch
    with torch.no_grad():
        cT = download(*AG.split_steps(p, seq, steps, m0, h0))
    w = O.mode_weights(2, prob.k)[:, None]
    S = vol * float(np.sum(w * np.abs(cT - tgt) * np.abs(cT)))
    nsw = steps * len(seq)
    worst = 0.0
    for d in dirs:
        Lp = _loss_only(sl, p, seq, steps, c0 + h * d, tgt, vol)
        Lm = _loss_only(sl, p, seq, steps, c0 - h * d, tgt, vol)
        fd = (Lp - Lm) / (2 * h)
        gd = math.fsum((g * d).ravel().tolist())
        tol = 2 * nsw * eps * S / h + 1e-10 * abs(gd)
        worst = max(worst, abs(fd - gd) / tol)
        assert abs(fd - gd) <= tol, (fd, gd, tol)
    print(f"finite differences n={n}: worst error / bound = {worst:.3f}")


def test_frozen_field_gradient_is_the_transpose_of_the_sweeps_run(sl):
    """With displacements computed from the state at the start of each step
    (the self-consistent field of section II), the gradient holds them fixed:
    it must equal the transposed sweeps, in reverse order, with exactly the
    displacements the forward pass used, and must not depend on
    checkpointing (the fields are rebuilt bitwise from the checkpoints)."""
    import torch
    from paper_1603_07008_amd import autograd as AG
    prob = inputs.landau_2d(32, 24, 2, 0.2, 0.5, eps=0.05)
    hx, hv = prob.h
    p = sl.Plan(prob.ns, prob.k, "fp64")
    sx = _dev(prob.seq[0].sigma)
    recorded = []

    def fields(state):
        sv = p.poisson_shift(state[0], state[1], hx, hv, prob.dt)
        recorded.append(sv.clone())
        return [(0, 2, sx), (1, 1, sv), (0, 2, sx)]

    c0 = O.project_separable(prob.f0_terms, prob.ns, prob.los, prob.his, prob.k)
    m0, h0 = upload(c0, "fp64")
    rng = np.random.default_rng(3)
    tm = _dev(c0[0] + 1e-3 * rng.standard_normal(c0.shape[1]))
    th = _dev(c0[1:] + 1e-3 * rng.standard_normal(c0[1:].shape))
    steps, vol = 6, hx * hv
    grads = {}
    for ckpt in (None, 2):
        recorded.clear()
        mm = m0.clone().requires_grad_(True)
        hh = h0.clone().requires_grad_(True)
        fm, fh = AG.split_steps(p, None, steps, mm, hh, checkpoint_every=ckpt,
                                frozen_shifts_fn=fields)
        loss = AG.weighted_l2_misfit(fm, fh, tm, th, 2, prob.k, vol)
        loss.backward()
        grads[ckpt] = (mm.grad.clone(), hh.grad.clone())
        if ckpt is None:
            fields_used = [r.clone() for r in recorded]
            final = (fm.detach().clone(), fh.detach().clone())
    assert len(fields_used) == steps
    for a, b in zip(grads[None], grads[2]):
        assert torch.equal(a, b)
    # the transposed sweeps with the recorded fields, from the loss gradient
    w = O.mode_weights(2, prob.k)
    g = (vol * w[0] * (final[0] - tm),
         (vol * torch.from_numpy(w[1:, None]).cuda() * (final[1] - th)).contiguous())
    tmp = p.empty_state()
    for n in range(steps - 1, -1, -1):
        for dim, mask, sh in reversed([(0, 2, sx), (1, 1, fields_used[n]), (0, 2, sx)]):
            p.advect_dim_adjoint(dim, sh, mask, g[0], g[1], tmp[0], tmp[1])
            g, tmp = tmp, g
    want = download(*g)
    got = download(*grads[None])
    scale = np.max(np.abs(want))
    assert np.max(np.abs(got - want)) <= 1e-13 * scale
    # and the fields really changed from step to step (a self-consistent run)
    assert not torch.equal(fields_used[0], fields_used[-1])
