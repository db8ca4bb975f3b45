"""GPU parity of the strided sweep staged through LDS (column waves plus
SLDG_SHAPE_STAGED): a workgroup loads its tile's source rows with 16-byte
accesses and each thread reads its own column from LDS with its own shift;
with SLDG_SHAPE_MEMORDER the tiles (staged or direct) go in memory order.
The arithmetic of every output is the direct strided kernel's, so the staged
sweep must give the direct sweep's bits on every cell (section II-A update
out[i] = A in[i-s] + B in[i-s-1]); one sweep per case is also held to the
oracle with the element-wise bound of the arithmetic.

Displacement fields: a narrow one whose integer shifts wrap around the period
inside a tile (s = N-1 next to s = 0), a smooth one whose per-tile spread is
sometimes larger than the LDS tile holds (those tiles take the direct path
inside the same launch), and a wide one (every tile direct).  Grids where
the staged form does not apply (column runs shorter than a tile, ragged row
tiles) must run the direct kernel under the staged shape.
"""
import zlib

import numpy as np
import pytest

from oracle import sldg_oracle as O
from paper_1603_07008_amd import inputs
from gpu_helpers import assert_sweep_close, download_nd, have_gpu, upload_nd

pytestmark = pytest.mark.gpu

SHAPES = [(4, 1), (4, 2), (8, 1), (8, 2), (4, 4), (8, 4)]   # (rows per thread, column waves)

# (extents, degree, swept dim, dimensions the displacement depends on)
CASES = [
    ((32, 4, 32, 16), 2, 2, (0, 1)),
    ((32, 4, 32, 16), 2, 3, (0, 1)),
    ((32, 4, 32, 16), 1, 2, (0, 1, 3)),
    ((32, 4, 16, 32), 3, 3, (0, 1)),
]


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


def _field(kind, ns, dep, rng):
    """Displacements (in cells) on the dep dimensions, dimension 0 fastest."""
    shape = [ns[e] for e in dep]
    n = int(np.prod(shape))
    if kind == "narrow":
        return rng.uniform(-1.5, 1.5, n)
    if kind == "wide":
        return rng.uniform(-40.0, 40.0, n)
    # smooth: a few cells of drift along the first dep dimension, plus noise
    x = (np.arange(n) % shape[0]) / shape[0]
    return 6.0 * np.sin(2 * np.pi * x) + rng.uniform(-0.5, 0.5, n)


def _expected_form(ns, k, dim, tier, rows, cw):
    """Whether the staged kernel applies (the host's rule, restated)."""
    P = int(np.prod(ns[:dim]))
    N = ns[dim]
    sz = {"fp32": 4, "bf16": 2, "fp16": 2}[tier]
    ch = 64 * cw // (16 // sz)
    rt = (4 // cw) * rows
    slots = ((k + 1) * (rt + 1) * ch + 255) // 256 + (1 if sz == 2 else 0)
    if cw == 4:
        slots = max(slots, ((k + 1) * (rt + 3) * ch + 255) // 256)
    umax = slots * 256 // ((k + 1) * ch)
    lds = 2 * (k + 1) * umax * 64 * cw * sz
    cells = int(np.prod(ns))
    extent = ((k) * (k + 1) ** dim + 1) * cells * sz
    ok = (P % (64 * cw) == 0 and N % ((4 // cw) * rows) == 0 and lds <= 64 * 1024
          and extent < 2 ** 31)
    return "staged" if ok else "strided"


@pytest.mark.parametrize("tier", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("field", ["narrow", "smooth", "wide"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{'x'.join(map(str, c[0]))}-k{c[1]}-d{c[2]}")
def test_staged_sweep_is_bitwise_the_direct_sweep(sl, case, field, tier):
    import torch
    ns, k, dim, dep = case
    ndim = len(ns)
    cells = int(np.prod(ns))
    rng = np.random.default_rng(zlib.crc32(repr(("staged", ns, k, dim, field, tier)).encode()))
    state = O.to_tier(inputs.random_coefficients(ndim, k, cells, seed=int(rng.integers(1 << 30))),
                      tier, k=k, ndim=ndim)
    sig = _field(field, ns, dep, rng)
    mask = sum(1 << e for e in dep)
    p = sl.Plan(ns, k, tier)
    s_in = upload_nd(state, p)
    shift = _dev(sig)
    checked = False
    nstaged = 0
    for rows, cw in SHAPES:
        for tuples in (3, 0):
            outs = []
            flags = (0, sl.SLDG_SHAPE_STAGED, sl.SLDG_SHAPE_MEMORDER,
                     sl.SLDG_SHAPE_STAGED | sl.SLDG_SHAPE_MEMORDER)
            for flag in flags:
                p.set_shape(dim, rows, tuples, cw | flag)
                s_out = p.empty_state()
                s_out[0].fill_(float("nan"))      # a cell left unwritten fails
                s_out[1].fill_(float("nan"))
                form = p.sweep_form(dim, mask, s_in, s_out)
                staged = flag & sl.SLDG_SHAPE_STAGED
                want_form = _expected_form(ns, k, dim, tier, rows, cw) if staged else "strided"
                assert form == want_form, (rows, cw, flag, form)
                nstaged += form == "staged"
                p.advect_dim(dim, shift, mask, s_in[0], s_in[1], s_out[0], s_out[1])
                outs.append(s_out)
            torch.cuda.synchronize()
            iview = torch.int16 if tier != "fp32" else torch.int32
            for flag, o in zip(flags[1:], outs[1:]):
                what = (f"{ns} k={k} d={dim} {tier} {field} rows={rows} cw={cw} tuples={tuples} "
                        f"flags={flag}")
                assert torch.equal(outs[0][0], o[0]), what + ": mass differs"
                assert torch.equal(outs[0][1].view(iview), o[1].view(iview)), \
                    what + ": differs from the direct sweep in the default order"
            if not checked:
                got = download_nd(outs[1][0], outs[1][1], p)
                want = O.sweep(state, ns, k, dim, sig, dep, tier)
                mag = O.sweep(state, ns, k, dim, sig, dep, absolute=True)
                keep = O.fp64_modes(ndim, k).astype(bool)
                assert_sweep_close(got, want, mag, tier, k, keep=keep, what=what)
                checked = True
    assert nstaged > 0
    p.close()


def test_staged_shape_on_grids_it_does_not_fit_runs_direct(sl):
    """Column runs shorter than a tile (P % 64 != 0) and ragged row tiles:
    the staged request runs the direct kernel, with the direct bits."""
    import torch
    for ns, dim in (((48, 5, 24), 1), ((64, 4, 20), 2)):
        k, tier = 2, "bf16"
        ndim = len(ns)
        cells = int(np.prod(ns))
        state = O.to_tier(inputs.random_coefficients(ndim, k, cells, seed=5), tier, k=k, ndim=ndim)
        p = sl.Plan(ns, k, tier)
        s_in = upload_nd(state, p)
        sig = np.random.default_rng(3).uniform(-3, 3, ns[0])
        outs = []
        for cw in (1, 1 | sl.SLDG_SHAPE_STAGED):
            p.set_shape(dim, 8, 0, cw)
            s_out = p.empty_state()
            assert p.sweep_form(dim, 1, s_in, s_out) == "strided"
            p.advect_dim(dim, _dev(sig), 1, s_in[0], s_in[1], s_out[0], s_out[1])
            outs.append(s_out)
        torch.cuda.synchronize()
        assert torch.equal(outs[0][1].view(torch.int16), outs[1][1].view(torch.int16))
        assert torch.equal(outs[0][0], outs[1][0])
        p.close()
