"""Guard-band canaries around every buffer a kernel writes.

Each output buffer sits inside a larger allocation whose bytes before and
after it (4 KiB each side, so 16-byte alignment is kept) hold a fill pattern;
every input buffer is guarded the same way.  Each case runs twice, with two
different fill patterns in the outputs, and checks that
  - the guard bytes of every output still hold the fill (no write outside
    the buffer), and no byte of any input allocation changed;
  - the two runs' outputs are bitwise equal (an element the kernel did not
    write would still hold the fill, which differs between the runs).
Forms covered: the window, group and lane forms along dimension 0, the
strided kernel over rows 1/2/4/8, tuple runs and column-wave layouts, the
lane form along strided dimensions, the kernels with leading FP64 modes,
every storage tier, the scaled FP16 sweep including the repair of a plane
that outgrows its headroom (scale blocks guarded too), the Gauss-node
collocated sweep, every class of the batched sweep, the (x, v) and
(x1, x2, v1, v2) field solves, the adjoint and the device mass.  Results
themselves are checked against the oracle elsewhere."""
import numpy as np
import pytest

from oracle import sldg_oracle as O
from paper_1603_07008_amd import inputs
from gpu_helpers import have_gpu

pytestmark = pytest.mark.gpu

GUARD = 4096
FILLS = (0xA5, 0x5A)
IN_FILL = 0xC3


@pytest.fixture(scope="module")
def sl():
    if not have_gpu():
        pytest.skip("no HIP device")
    import paper_1603_07008_amd as sl
    sl.lib()
    return sl


class Guarded:
    """A buffer of `n` elements of `dtype` between two guard bands."""

    def __init__(self, n, dtype, fill):
        import torch
        item = torch.empty((), dtype=dtype).element_size()
        self.g = GUARD // item
        self.n = int(n)
        self.fill = fill
        self.full = torch.empty(self.n + 2 * self.g, dtype=dtype, device="cuda")
        self.full.view(torch.uint8).fill_(fill)
        self.view = self.full[self.g:self.g + self.n]

    def guards_hold(self):
        import torch
        b = self.full.view(torch.uint8)
        gb = self.g * self.full.element_size()
        nb = self.n * self.full.element_size()
        return bool(torch.all(b[:gb] == self.fill)) and bool(torch.all(b[gb + nb:] == self.fill))

    def bytes(self):
        import torch
        return self.view.view(torch.uint8).clone()


def guarded_input(t):
    g = Guarded(t.numel(), t.dtype, IN_FILL)
    g.view.copy_(t.reshape(-1))
    return g


def run_guarded(make_inputs, out_specs, op):
    """make_inputs() -> list of device tensors (copied into guarded buffers);
    out_specs: [(n, dtype)]; op(inputs, outputs) launches the kernels."""
    import torch
    runs = []
    for fill in FILLS:
        ins = [guarded_input(t) for t in make_inputs()]
        before = [g.full.view(torch.uint8).clone() for g in ins]
        outs = [Guarded(n, dt, fill) for n, dt in out_specs]
        op([g.view for g in ins], [g.view for g in outs])
        torch.cuda.synchronize()
        for i, g in enumerate(outs):
            assert g.guards_hold(), f"output {i}: a guard byte changed (fill {fill:#x})"
        for i, (g, b) in enumerate(zip(ins, before)):
            assert torch.equal(g.full.view(torch.uint8), b), f"input {i} changed"
        runs.append([g.bytes() for g in outs])
    for i, (a, b) in enumerate(zip(*runs)):
        assert torch.equal(a, b), f"output {i}: some elements were not written"


def state_inputs(sl, plan, seed):
    import torch
    ndim = len(plan.ncells)
    m, h = inputs.random_coefficients_device(ndim, plan.k, plan.cells, seed=seed)
    if plan.n_lo == 1:
        return m.contiguous(), h.to(sl.hi_dtype(plan.tier)).contiguous()
    # leading FP64 modes beyond the mean: take them from the narrow planes
    full = torch.cat([m[None], h], 0)
    pm = plan.plane_map()
    lo = [mm for _, mm in sorted((-1 - v, mm) for mm, v in enumerate(pm) if v < 0)]
    hi = [mm for _, mm in sorted((v, mm) for mm, v in enumerate(pm) if v >= 0)]
    return full[lo].contiguous(), full[hi].to(sl.hi_dtype(plan.tier)).contiguous()


def state_specs(sl, plan):
    import torch
    return [(plan.n_lo * plan.cells, torch.float64), (plan.n_hi * plan.cells, sl.hi_dtype(plan.tier))]


def shift_for(plan, dep, seed, spread=2.5):
    import torch
    n = 1
    for e in dep:
        n *= plan.ncells[e]
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.uniform(-spread, spread, n)).cuda()


def mask_of(dep):
    return sum(1 << e for e in dep)


# ---------------------------------------------------------------------------

# (grid, dim, dep, shape (rows, tuples, colwaves) or None for the default)
SWEEPS = [
    ((36, 7), 0, (1,), None),               # window form
    ((36, 7), 0, (), (0, 3, 1)),            # window form, tuple runs of 3
    ((37, 7), 0, (1,), None),               # group form (displacement depends on dim 1)
    ((37, 7), 0, (1,), (4, 2, 1)),
    ((37, 7), 0, (), None),                 # lane form (automatic)
    ((37, 7), 0, (1,), (1, 0, 1)),          # lane form (asked for)
    ((37, 13, 5), 1, (0,), (1, 1, 1)),      # strided, one row per thread
    ((37, 13, 5), 1, (0,), (2, 3, 2)),
    ((37, 13, 5), 1, (0, 2), (4, 0, 4)),
    ((37, 13, 5), 1, (2,), (8, 9, 1)),      # 13 rows: a ragged last chunk of 8
    ((37, 13, 5), 2, (0, 1), (8, 1, 2)),
    ((37, 13, 5), 2, (0, 1), (0, 3, 1)),    # lane form along a strided dimension
    ((64, 3, 6), 2, (1,), (4, 9, 1)),       # P % 64 == 0: non-temporal stores
]


@pytest.mark.parametrize("tier", ["fp64", "fp32", "bf16", "fp16"])
@pytest.mark.parametrize("case", range(len(SWEEPS)))
def test_sweep_forms_write_exactly_their_outputs(sl, tier, case):
    ns, dim, dep, shape = SWEEPS[case]
    plan = sl.Plan(ns, 2, tier)
    if shape is not None:
        plan.set_shape(dim, *shape)
    sig = shift_for(plan, dep, 100 + case)
    run_guarded(lambda: list(state_inputs(sl, plan, 200 + case)), state_specs(sl, plan),
                lambda i, o: plan.advect_dim(dim, sig, mask_of(dep), *i, *o))
    run_guarded(lambda: list(state_inputs(sl, plan, 300 + case)), state_specs(sl, plan),
                lambda i, o: plan.advect_dim_adjoint(dim, sig, mask_of(dep), *i, *o))
    plan.close()


@pytest.mark.parametrize("k", [1, 3])
@pytest.mark.parametrize("case", [0, 2, 4, 8, 10])
def test_leading_fp64_mode_kernels_write_exactly_their_outputs(sl, k, case):
    ns, dim, dep, shape = SWEEPS[case]
    plan = sl.Plan(ns, k, "fp32", ndouble=2)
    if shape is not None:
        plan.set_shape(dim, *shape)
    sig = shift_for(plan, dep, 400 + case)
    run_guarded(lambda: list(state_inputs(sl, plan, 500 + case)), state_specs(sl, plan),
                lambda i, o: plan.advect_dim(dim, sig, mask_of(dep), *i, *o))
    plan.close()


@pytest.mark.parametrize("tier", ["fp64", "fp32", "bf16", "fp16"])
def test_fused_pair_writes_exactly_its_outputs(sl, tier):
    for ns, rows in (((48, 13, 5), "0"), ((12, 7, 3, 2), "3")):
        import os
        old = os.environ.get("SLDG_XY_ROWS")
        os.environ["SLDG_XY_ROWS"] = rows
        try:
            plan = sl.Plan(ns, 2, tier)
        finally:
            if old is None:
                os.environ.pop("SLDG_XY_ROWS")
            else:
                os.environ["SLDG_XY_ROWS"] = old
        s0 = shift_for(plan, (2,), 60)
        s1 = shift_for(plan, (2,), 61)
        run_guarded(lambda: list(state_inputs(sl, plan, 62)), state_specs(sl, plan),
                    lambda i, o: plan.advect_dims01(s0, 4, s1, 4, *i, *o))
        plan.close()


def test_scaled_fp16_sweep_and_repair_write_exactly_their_outputs(sl):
    import torch
    from test_gpu_scaled import upload_scaled
    n0, n1, k = 64, 9, 2
    rng = np.random.default_rng(7)
    st = np.zeros(((k + 1) ** 2, n0 * n1))
    cells = np.arange(n0 * n1)
    st[0] = np.where(cells % n0 < n0 // 2, 1.0, 0.25)        # a step: planes outgrow headroom
    st[1:] = 1e-12 * rng.standard_normal((st.shape[0] - 1, st.shape[1]))
    plan = sl.Plan((n0, n1), k, "fp16")
    m, h, s = upload_scaled(plan, O.to_scaled(st, k, 2))
    specs = state_specs(sl, plan) + [(2 * plan.n_hi, torch.int32)]
    for dim, dep in ((0, (1,)), (1, (0,))):
        sig = torch.from_numpy(np.full(plan.ncells[dep[0]], 0.3)).cuda()
        run_guarded(lambda: [m, h, s], specs,
                    lambda i, o: plan.advect_dim_scaled(dim, sig, mask_of(dep), *i, *o))
    # plain scaled sweeps of random data along a strided dimension of a 3D grid
    p3 = sl.Plan((37, 13, 5), k, "fp16")
    st3 = inputs.random_coefficients(3, k, p3.cells, seed=11)
    m3, h3, s3 = upload_scaled(p3, O.to_scaled(st3, k, 3))
    p3.set_shape(1, 4, 3, 2)
    sig3 = shift_for(p3, (0,), 12)
    run_guarded(lambda: [m3, h3, s3], state_specs(sl, p3) + [(2 * p3.n_hi, torch.int32)],
                lambda i, o: p3.advect_dim_scaled(1, sig3, 1, *i, *o))
    plan.close()
    p3.close()


def test_collocated_sweep_writes_exactly_its_outputs(sl):
    import torch
    for ns, dim, t in (((37, 11), 0, 1), ((36, 11, 3), 1, 0), ((64, 5, 4), 0, 2)):
        plan = sl.Plan(ns, 2, "fp32")
        rng = np.random.default_rng(13)
        node = torch.from_numpy(rng.uniform(-3, 3, ns[t] * 3)).cuda()
        run_guarded(lambda: list(state_inputs(sl, plan, 14)), state_specs(sl, plan),
                    lambda i, o: plan.advect_dim_collocated(dim, t, node, *i, *o))
        plan.close()


def test_batched_classes_write_exactly_their_outputs(sl):
    import torch
    from paper_1603_07008_amd.batch import Batch
    ns = [(36, 20), (37, 21), (33, 9), (64, 17), (40, 3)]
    ks = [1, 2, 3, 2, 3]
    for dim in (0, 1):
        for rows in ((4, 1) if dim == 0 else (2, 4, 8, 0)):
            b = Batch(ns, ks, "fp32")
            per = []
            for p, (n, k) in enumerate(zip(ns, ks)):
                dep = (1 - dim,)
                per.append((mask_of(dep), torch.from_numpy(
                    np.random.default_rng(p).uniform(-2.5, 2.5, n[1 - dim])).cuda()))

            def make_inputs():
                out = []
                for p, (n, k) in enumerate(zip(ns, ks)):
                    m, h = inputs.random_coefficients_device(2, k, n[0] * n[1], seed=30 + p)
                    out += [m, h.to(torch.float32).contiguous()]
                return out
            specs = []
            for n, k in zip(ns, ks):
                specs += [(n[0] * n[1], torch.float64), (((k + 1) ** 2 - 1) * n[0] * n[1],
                                                          torch.float32)]

            def op(i, o):
                b.bind([(i[2 * p], i[2 * p + 1]) for p in range(len(ns))],
                       [(o[2 * p], o[2 * p + 1]) for p in range(len(ns))])
                b.set_sequence([(dim, per)])
                for cls in range(9):
                    if cls // 3 == (2 if dim else 0) or (dim == 0 and cls // 3 == 1):
                        r = rows if cls // 3 != 0 else 4
                        b.set_class_tuning(0, cls, r, 3)
                assert b.run(1) == 1
            run_guarded(make_inputs, specs, op)
            b.close()


def test_field_solves_and_mass_write_exactly_their_outputs(sl):
    import torch
    plan = sl.Plan((37, 23), 2, "fp32")
    n = plan.ncells[0]
    run_guarded(lambda: list(state_inputs(sl, plan, 40)),
                [(n, torch.float64), (n, torch.float64)],
                lambda i, o: plan.poisson_shift(*i, 0.37, 0.21, 0.1, shift_out=o[0],
                                                field_out=o[1]))
    run_guarded(lambda: list(state_inputs(sl, plan, 41)),
                [(n, torch.float64), (n, torch.float64)],
                lambda i, o: plan.poisson_shift_noalloc(*i, 0.37, 0.21, 0.1, shift_out=o[0],
                                                        field_out=o[1]))
    run_guarded(lambda: list(state_inputs(sl, plan, 42))[:1], [(2, torch.float64)],
                lambda i, o: plan.mass_device(i[0], o[0]))
    plan.close()
    p4 = sl.Plan((12, 10, 6, 5), 1, "fp32")
    nxx = 12 * 10
    run_guarded(lambda: list(state_inputs(sl, p4, 43)),
                [(nxx, torch.float64), (nxx, torch.float64), (2 * nxx, torch.float64)],
                lambda i, o: p4.poisson_shift_2d(*i, (0.37, 0.29, 0.21, 0.17), 0.1,
                                                 shift_v1=o[0], shift_v2=o[1], field_out=o[2]))
    p4.close()
