"""Batched sweeps: every problem of a batch matches its own single-problem
run bit for bit (same kernels, same arithmetic) and the oracle; graph replays
match eager runs; tuning changes speed, not results."""
import numpy as np
import pytest

from oracle import sldg_oracle as O
from paper_1603_07008_amd import inputs
from gpu_helpers import download, have_gpu, upload, weighted_rel_l2

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


def _problems():
    probs = inputs.batched_landau(nprob=9, seed=11, nmin=17, nmax=70)
    probs.append(inputs.landau_2d(64, 40, 2, 0.1, 0.5))     # window path (N0 % 4 == 0)
    probs.append(inputs.landau_2d(33, 8, 3, 0.15, 0.7))     # generic path
    return probs


def _setup(sl, probs, tier, stream):
    from paper_1603_07008_amd.batch import Batch
    b = Batch([p.ns for p in probs], [p.k for p in probs], tier, stream=stream)
    c0s = [O.to_tier(O.project_separable(p.f0_terms, p.ns, p.los, p.his, p.k), tier) for p in probs]
    s0 = [upload(c, tier) for c in c0s]
    s1 = [(m.clone(), h.clone()) for m, h in s0]
    b.bind(s0, s1)
    shifts = [[(sw.dep_mask, _dev(sw.sigma)) for sw in p.seq] for p in probs]
    seq = [(probs[0].seq[q].dim, [shifts[p][q] for p in range(len(probs))]) for q in range(3)]
    b.set_sequence(seq)
    return b, c0s, s0, s1, shifts


@pytest.mark.parametrize("tier", ["fp64", "fp32", "bf16"])
def test_batch_matches_single_problem_runs_and_oracle(sl, tier):
    import torch
    probs = _problems()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b, c0s, s0, s1, shifts = _setup(sl, probs, tier, stream.cuda_stream)
        steps = 3
        res = b.run(steps)
        stream.synchronize()
        for i, p in enumerate(probs):
            got = download(*(s0, s1)[res][i])
            plan = sl.Plan(p.ns, p.k, tier, stream=stream.cuda_stream)
            a = upload(c0s[i], tier)
            c = plan.empty_state()
            r = plan.split_steps([(sw.dim, sw.dep_mask, shifts[i][q][1]) for q, sw in enumerate(p.seq)],
                                 steps, a, c)
            stream.synchronize()
            single = download(*(a, c)[r])
            assert np.array_equal(got, single), (i, p.ns, p.k)
            want = O.run_sequence(c0s[i], p.ns, p.k, [(s.dim, s.sigma, s.dep) for s in p.seq],
                                  tier, steps)
            tol = {"fp64": 1e-13, "fp32": 2.0 ** -24, "bf16": 1e-3}[tier]
            assert weighted_rel_l2(got, want, 2, p.k) <= tol


def test_graph_replays_match_eager_and_tuning_keeps_results(sl):
    import torch
    probs = _problems()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b, c0s, s0, s1, shifts = _setup(sl, probs, "fp32", stream.cuda_stream)
        init = [(m.clone(), h.clone()) for m, h in s0]
        # eager reference: 4 steps, result after each step
        ref = []
        for n in range(4):
            res = b.run(1)
            stream.synchronize()
            ref.append([download(*(s0, s1)[res][i]) for i in range(len(probs))])
            if res == 1:        # move the state back to buffer 0 for the next step
                for i in range(len(probs)):
                    s0[i][0].copy_(s1[i][0])
                    s0[i][1].copy_(s1[i][1])
        # graph replays from the same start, with eager work in between
        for i in range(len(probs)):
            s0[i][0].copy_(init[i][0])
            s0[i][1].copy_(init[i][1])
        stream.synchronize()
        for n in range(4):
            res = b.run(1, use_graph=True)
            stream.synchronize()
            for i in range(len(probs)):
                assert np.array_equal(download(*(s0, s1)[res][i]), ref[n][i]), (n, i)
            torch.cuda.synchronize()
            if res == 1:
                for i in range(len(probs)):
                    s0[i][0].copy_(s1[i][0])
                    s0[i][1].copy_(s1[i][1])
        # tuning (clobbers buffer 1) then one step from the initial state again
        shapes = b.tune(reps=2)
        assert len(shapes) == 3 and all(s["ms"] > 0 for s in shapes)
        for i in range(len(probs)):
            s0[i][0].copy_(init[i][0])
            s0[i][1].copy_(init[i][1])
        res = b.run(1)
        stream.synchronize()
        for i in range(len(probs)):
            assert np.array_equal(download(*(s0, s1)[res][i]), ref[0][i])


@pytest.mark.parametrize("tier", ["fp32", "bf16"])
def test_batch_lane_and_tiled_forms_agree_bitwise(sl, tier):
    """The lane form (rows 1 for the non-window dimension-0 classes, rows 0
    for the strided classes) and the tiled forms (4-cell groups, 8 rows per
    thread), with one tuple or all per thread, give the same bits on every
    cell (the second buffer starts as NaN)."""
    import torch
    probs = _problems()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b, c0s, s0, s1, shifts = _setup(sl, probs, tier, stream.cuda_stream)
        init = [(m.clone(), h.clone()) for m, h in s0]
        ref = None
        for rows, vrows in ((4, 8), (1, 0), (4, 0)):
            for tuples in (1, 0):
                for q in (0, 2):                       # the two x-sweeps of the step
                    for cls in (3, 4, 5):              # dimension-0 group classes, k = 1..3
                        b.set_class_tuning(q, cls, rows, tuples)
                for cls in (6, 7, 8):                  # strided classes of the v-sweep
                    b.set_class_tuning(1, cls, vrows, tuples)
                for i in range(len(probs)):
                    s0[i][0].copy_(init[i][0])
                    s0[i][1].copy_(init[i][1])
                    s1[i][0].fill_(float("nan"))
                    s1[i][1].fill_(float("nan"))
                res = b.run(2)
                stream.synchronize()
                got = [download(*(s0, s1)[res][i]) for i in range(len(probs))]
                if ref is None:
                    ref = got
                else:
                    for i in range(len(probs)):
                        assert np.array_equal(got[i], ref[i]), (rows, tuples, i)
        assert any(p.ns[0] % 4 for p in probs)


def test_full_batched_workload_matches_single_plans_and_oracle(sl):
    """The batched workload at its full size (512 problems, N_x, N_v in
    32..512, k in 1..3, FP32-mode) in the launch shapes the batch tuner
    picks: every problem bitwise equal to its own single-plan run, a sample
    against the oracle."""
    import torch
    probs = inputs.batched_landau(nprob=512, seed=4)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        from paper_1603_07008_amd.batch import Batch
        b = Batch([p.ns for p in probs], [p.k for p in probs], "fp32", stream=stream.cuda_stream)
        c0s = [O.to_tier(inputs.random_coefficients(2, p.k, p.cells, seed=100 + i), "fp32")
               for i, p in enumerate(probs)]
        s0 = [upload(c, "fp32") for c in c0s]
        s1 = [(m.clone(), h.clone()) for m, h in s0]
        b.bind(s0, s1)
        shifts = [[(sw.dep_mask, _dev(sw.sigma)) for sw in p.seq] for p in probs]
        b.set_sequence([(probs[0].seq[q].dim, [shifts[i][q] for i in range(len(probs))])
                        for q in range(3)])
        b.tune(reps=1)
        for i in range(len(probs)):            # start from the initial state again
            m, h = upload(c0s[i], "fp32")
            s0[i][0].copy_(m)
            s0[i][1].copy_(h)
        res = b.run(1, use_graph=True)
        stream.synchronize()
        rng = np.random.default_rng(12)
        sample = set(rng.choice(len(probs), 6, replace=False).tolist())
        for i, p in enumerate(probs):
            got = download(*(s0, s1)[res][i])
            plan = sl.Plan(p.ns, p.k, "fp32", stream=stream.cuda_stream)
            a = upload(c0s[i], "fp32")
            c = plan.empty_state()
            r = plan.split_steps([(sw.dim, sw.dep_mask, shifts[i][q][1])
                                  for q, sw in enumerate(p.seq)], 1, a, c)
            stream.synchronize()
            assert np.array_equal(got, download(*(a, c)[r])), (i, p.ns, p.k)
            plan.close()
            if i in sample:
                want = O.run_sequence(c0s[i], p.ns, p.k, [(s.dim, s.sigma, s.dep) for s in p.seq],
                                      "fp32", 1)
                assert weighted_rel_l2(got, want, 2, p.k) <= 2.0 ** -24, (i, p.ns, p.k)
        b.close()
