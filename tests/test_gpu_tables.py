"""Split steps compute the line tables of their whole sweep sequence in one
launch before the steps (the displacements are fixed over a call), where the
sequence's tables fit the plan's table storage together and the sequence has
at most 16 sweeps; otherwise each sweep computes its own.  Either way a split
step must give the bits of the same sweeps called one at a time (section II:
the split step is the composition of the one-dimensional sweeps)."""
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


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _run_both(sl, ns, k, tier, seq, nsteps, seed):
    import torch
    ndim = len(ns)
    cells = int(np.prod(ns))
    state = O.to_tier(inputs.random_coefficients(ndim, k, cells, seed=seed), tier)
    plan = sl.Plan(ns, k, tier)
    plan.set_fusion(False)
    dseq = [(d, mask, _dev(sig)) for d, mask, sig in seq]
    a = upload(state, tier)
    b = plan.empty_state()
    r = plan.split_steps(dseq, nsteps, a, b)
    torch.cuda.synchronize()
    got = download(*(a, b)[r])
    # the same sweeps, one call each
    bufs = [upload(state, tier), plan.empty_state()]
    cur = 0
    for _ in range(nsteps):
        for d, mask, sig in dseq:
            plan.advect_dim(d, sig, mask, *bufs[cur], *bufs[1 - cur])
            cur = 1 - cur
    torch.cuda.synchronize()
    want = download(*bufs[cur])
    plan.close()
    return got, want


@pytest.mark.parametrize("tier", ["fp64", "fp32", "bf16"])
def test_split_steps_with_one_table_launch_match_single_sweeps(sl, tier):
    ns, k = (40, 24, 12), 2
    rng = np.random.default_rng(5)
    seq = [(0, 0b010, rng.uniform(-9, 9, ns[1])), (1, 0b100, rng.uniform(-5, 5, ns[2])),
           (2, 0b001, rng.uniform(-3, 3, ns[0])), (0, 0b010, rng.uniform(-9, 9, ns[1]))]
    got, want = _run_both(sl, ns, k, tier, seq, 3, 11)
    assert np.array_equal(got, want)


def test_split_steps_longer_than_one_table_launch_match_single_sweeps(sl):
    ns, k = (36, 20), 1
    rng = np.random.default_rng(6)
    seq = [(q % 2, 0b10 if q % 2 == 0 else 0b01, rng.uniform(-7, 7, ns[1 - q % 2]))
           for q in range(19)]
    got, want = _run_both(sl, ns, k, "fp32", seq, 2, 12)
    assert np.array_equal(got, want)


def test_split_steps_whose_tables_exceed_the_storage_match_single_sweeps(sl):
    # every sweep's displacement depends on both other dimensions: each table
    # has cells / N_d entries, and the sequence's tables together exceed the
    # plan's storage (the largest single table)
    ns, k = (24, 16, 10), 2
    rng = np.random.default_rng(7)
    cells = int(np.prod(ns))
    seq = [(d, 0b111 & ~(1 << d), rng.uniform(-6, 6, cells // ns[d])) for d in (0, 1, 2, 1)]
    got, want = _run_both(sl, ns, k, "fp32", seq, 2, 13)
    assert np.array_equal(got, want)
