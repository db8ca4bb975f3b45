"""The allocation-free field solve (sldg_poisson_shift_noalloc) against the
allocating one (sldg_poisson_shift), through the C ABI: the same kernels run
on a static device scratch array instead of a plan-owned buffer, so the
results must be bitwise equal.  Two calls in a row share the array, the
second on a smaller grid; a grid beyond the array's size is rejected before
anything is launched.  The fields are also held to the oracle (section II:
the field E(x) of the v-sweep)."""
import numpy as np
import pytest

from oracle import sldg_oracle as O
from paper_1603_07008_amd import inputs
from gpu_helpers import have_gpu, upload_nd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sl():
    if not have_gpu():
        pytest.skip("no HIP device")
    import paper_1603_07008_amd as sl
    sl.lib()
    return sl


def _both(sl, ns, k, tier, seed):
    import torch
    st = O.to_tier(inputs.random_coefficients(2, k, ns[0] * ns[1], seed=seed), tier)
    hx, hv, dt = 0.37, 0.21, 0.1
    plan = sl.Plan(ns, k, tier)
    m, h = upload_nd(st, plan)
    f_ref = torch.empty(ns[0], dtype=torch.float64, device="cuda")
    f_new = torch.full((ns[0],), float("nan"), dtype=torch.float64, device="cuda")
    s_ref = plan.poisson_shift(m, h, hx, hv, dt, field_out=f_ref)
    s_new = plan.poisson_shift_noalloc(m, h, hx, hv, dt, field_out=f_new)
    torch.cuda.synchronize()
    assert torch.equal(s_new, s_ref) and torch.equal(f_new, f_ref)
    want = O.poisson_field(st, ns, k, hx, hv)
    got = f_new.cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-12 * float(np.max(np.abs(want)))
    plan.close()


def test_noalloc_matches_allocating_entry_point_on_two_calls_in_a_row(sl):
    _both(sl, (3000, 24), 3, "fp32", 71)        # several scan chunks per thread
    _both(sl, (40, 16), 2, "bf16", 72)          # smaller grid on the same array


def test_noalloc_rejects_a_grid_beyond_the_static_scratch(sl):
    import torch
    ns, k = (15000, 8), 3                       # 37 * 15000 + 1 doubles > 2^19
    plan = sl.Plan(ns, k, "fp32")
    m, h = plan.empty_state()
    with pytest.raises(sl.SldgError) as ei:
        plan.poisson_shift_noalloc(m, h, 0.1, 0.1, 0.1)
    assert ei.value.status == sl.SLDG_ERR_UNSUPPORTED
    assert "static" in str(ei.value)
    plan.close()
