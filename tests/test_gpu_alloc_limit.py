"""Out-of-memory paths of the library, forced through its device allocation
limit (sldg_set_device_alloc_limit): every allocation the library makes for
itself (plan tables, scaled FP16 partials, field scratch, batch tables and
work lists) fails with SLDG_ERR_NOMEM when it would pass the limit, before any
kernel is launched, and leaves the plan or batch usable: with the limit
lifted the same call succeeds and gives bitwise the result of an unconstrained
run.  The limit is always lifted again, whatever the test's outcome."""
import numpy as np
import pytest

from oracle import sldg_oracle as O
from paper_1603_07008_amd import inputs
from gpu_helpers import have_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sl():
    if not have_gpu():
        pytest.skip("no HIP device")
    import paper_1603_07008_amd as sl
    sl.lib()
    return sl


@pytest.fixture
def limit(sl):
    """Sets a cap of (bytes held now + extra) while the test runs."""
    def set_extra(extra):
        sl.set_device_alloc_limit(sl.device_alloc_bytes() + int(extra))
    yield set_extra
    sl.set_device_alloc_limit(None)


def _nomem(sl, fn):
    with pytest.raises(sl.SldgError) as ei:
        fn()
    assert ei.value.status == sl.SLDG_ERR_NOMEM, ei.value


def test_plan_refused_and_nothing_leaks(sl, limit):
    held = sl.device_alloc_bytes()
    p = sl.Plan((64, 48), 2, "fp32")
    need = sl.device_alloc_bytes() - held
    assert need > 0
    p.close()
    assert sl.device_alloc_bytes() == held
    limit(need - 1)
    _nomem(sl, lambda: sl.Plan((64, 48), 2, "fp32"))
    assert sl.device_alloc_bytes() == held
    limit(need)
    q = sl.Plan((64, 48), 2, "fp32")
    q.close()
    assert sl.device_alloc_bytes() == held


def test_scaled_partials_nomem_then_recover(sl, limit):
    import torch
    ns, k = (40, 24), 2
    st = inputs.random_coefficients(2, k, 40 * 24, seed=3)
    hi64 = torch.from_numpy(np.ascontiguousarray(st[1:])).cuda()
    ref = sl.Plan(ns, k, "fp16")
    h_ref = torch.empty((ref.n_hi, ref.cells), dtype=torch.float16, device="cuda")
    s_ref = ref.empty_scale()
    ref.scaled_import(hi64, h_ref, s_ref)
    p = sl.Plan(ns, k, "fp16")
    h = torch.empty_like(h_ref)
    s = p.empty_scale()
    limit(0)
    _nomem(sl, lambda: p.scaled_import(hi64, h, s))
    sl.set_device_alloc_limit(None)
    p.scaled_import(hi64, h, s)
    torch.cuda.synchronize()
    assert torch.equal(h.view(torch.int16), h_ref.view(torch.int16))
    assert torch.equal(s, s_ref)
    # a scaled sweep that needs more partial slots than the import
    m = torch.from_numpy(np.ascontiguousarray(st[0])).cuda()
    sig = torch.from_numpy(np.full(ns[0], 0.3)).cuda()
    out_ref = (*ref.empty_state(), ref.empty_scale())
    ref.advect_dim_scaled(1, sig, 1, m, h_ref, s_ref, *out_ref)
    out = (*p.empty_state(), p.empty_scale())
    limit(0)
    try:
        p.advect_dim_scaled(1, sig, 1, m, h, s, *out)     # fits the import's buffer, or not
    except sl.SldgError as e:
        assert e.status == sl.SLDG_ERR_NOMEM
        sl.set_device_alloc_limit(None)
        p.advect_dim_scaled(1, sig, 1, m, h, s, *out)
    torch.cuda.synchronize()
    for a, b in zip(out, out_ref):
        assert torch.equal(a.view(torch.uint8), b.view(torch.uint8))
    p.close()
    ref.close()


def test_field_scratch_nomem_then_recover(sl, limit):
    import torch
    p = sl.Plan((48, 40), 2, "fp32")
    m, h = inputs.random_coefficients_device(2, 2, p.cells, seed=5)
    h = h.to(torch.float32).contiguous()
    want = O.poisson_field(np.concatenate([m.cpu().numpy()[None],
                                           h.double().cpu().numpy()]), (48, 40), 2, 0.37, 0.21)
    field = torch.empty(48, dtype=torch.float64, device="cuda")
    limit(0)
    _nomem(sl, lambda: p.poisson_shift(m, h, 0.37, 0.21, 0.1, field_out=field))
    # the allocation-free entry point needs no allocation
    p.poisson_shift_noalloc(m, h, 0.37, 0.21, 0.1, field_out=field)
    torch.cuda.synchronize()
    got_static = field.cpu().numpy().copy()
    sl.set_device_alloc_limit(None)
    p.poisson_shift(m, h, 0.37, 0.21, 0.1, field_out=field)
    torch.cuda.synchronize()
    got = field.cpu().numpy()
    assert np.array_equal(got, got_static)
    assert np.max(np.abs(got - want)) <= 1e-12 * float(np.max(np.abs(want)))
    p.close()


def test_batch_nomem_leaves_no_runnable_sequence(sl, limit):
    import torch
    from paper_1603_07008_amd.batch import Batch
    ns, ks = [(36, 20), (37, 21)], [1, 2]

    def states(seed):
        out = []
        for p, (n, k) in enumerate(zip(ns, ks)):
            m, h = inputs.random_coefficients_device(2, k, n[0] * n[1], seed=seed + p)
            out.append((m, h.to(torch.float32).contiguous()))
        return out

    seq = [(0, [(2, torch.from_numpy(np.linspace(-2, 2, n[1])).cuda()) for n in ns])]
    ref = Batch(ns, ks, "fp32")
    a0, a1 = states(10), [(torch.empty_like(m), torch.empty_like(h)) for m, h in states(10)]
    ref.bind(a0, a1)
    ref.set_sequence(seq)
    assert ref.run(1) == 1
    limit(0)
    _nomem(sl, lambda: Batch(ns, ks, "fp32"))
    sl.set_device_alloc_limit(None)
    b = Batch(ns, ks, "fp32")
    b0, b1 = states(10), [(torch.empty_like(m), torch.empty_like(h)) for m, h in states(10)]
    b.bind(b0, b1)
    limit(0)
    _nomem(sl, lambda: b.set_sequence(seq))
    with pytest.raises(sl.SldgError) as ei:
        b.run(1)                                   # no sequence: refused, nothing launched
    assert ei.value.status == sl.SLDG_ERR_ARG
    sl.set_device_alloc_limit(None)
    b.set_sequence(seq)
    assert b.run(1) == 1
    torch.cuda.synchronize()
    for (m, h), (rm, rh) in zip(b1, a1):
        assert torch.equal(m, rm) and torch.equal(h, rh)
    b.close()
    ref.close()
