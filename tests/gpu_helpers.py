"""Helpers shared by the GPU parity tests: moving states between the oracle's
FP64 layout and the library's split layout, and the element-wise error bound
derived from the arithmetic of the update."""
import math

import numpy as np

MANT = {"fp64": 52, "fp32": 23, "bf16": 7, "fp16": 10}
EMIN = {"fp64": -1022, "fp32": -126, "bf16": -126, "fp16": -14}


def have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def upload(state, tier):
    """Oracle state [M, cells] (FP64 values already representable in the tier)
    -> (mass, hi) device tensors in the library's layout."""
    import torch
    import paper_1603_07008_amd as sl
    mass = torch.from_numpy(np.ascontiguousarray(state[0], dtype=np.float64)).cuda()
    hi64 = torch.from_numpy(np.ascontiguousarray(state[1:], dtype=np.float64))
    hi = hi64.to(sl.hi_dtype(tier))
    assert torch.equal(hi.to(torch.float64), hi64), "state not representable in the tier"
    return mass, hi.cuda().contiguous()


def download(mass, hi):
    import torch
    m = mass.detach().to("cpu", torch.float64).numpy()
    h = hi.detach().to("cpu").to(torch.float64).numpy()
    return np.concatenate([m[None, :], h.reshape(-1, m.size)], axis=0)


def ulp(x, tier):
    """Spacing of the tier's format at |x| (gradual underflow below emin)."""
    ax = np.abs(np.asarray(x, dtype=np.float64))
    e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    e = np.where(ax > 0, np.maximum(e, EMIN[tier]), EMIN[tier])
    return np.ldexp(1.0, (e - MANT[tier]).astype(int))


def gamma(tier, k, mass_mode):
    """Bound on the relative accumulation error of one output of the update
    (2(k+1) products summed, matrices within an ulp of exact, and for the
    FP32-arithmetic tiers the matrices and the FP64 mass input rounded to FP32),
    relative to sum_l |A_jl x_l| + |B_jl y_l|."""
    n = 2 * (k + 1) + 4
    if mass_mode or tier in ("fp64", "fp32"):
        return 4 * n * 2.0 ** -53
    return n * 2.0 ** -24


def sweep_bound(want, got, mag, tier, k, keep=None):
    """Element-wise bound on |got - want| for one sweep from identical inputs:
    both sides round the exact update to the storage format, from values that
    differ by at most gamma * magnitude.  `keep` marks the FP64 modes (default:
    mode 0 alone)."""
    if keep is None:
        keep = np.zeros(want.shape[0], dtype=bool)
        keep[0] = True
    keep = np.asarray(keep, dtype=bool)
    tol = np.empty_like(want)
    big = np.maximum(np.abs(want), np.abs(got))
    tol[keep] = ulp(big[keep], "fp64") + gamma("fp64", k, True) * mag[keep]
    tol[~keep] = ulp(big[~keep], tier) + gamma(tier, k, False) * mag[~keep]
    return tol


def upload_nd(state, plan):
    """Oracle state -> (mass, hi) in the plan's layout for any number of FP64
    modes (plane map from the library)."""
    import torch
    import paper_1603_07008_amd as sl
    pm = plan.plane_map()
    lo = sorted((-1 - v, m) for m, v in enumerate(pm) if v < 0)
    hi = sorted((v, m) for m, v in enumerate(pm) if v >= 0)
    mass = torch.from_numpy(np.ascontiguousarray(state[[m for _, m in lo]])).cuda()
    if len(lo) == 1:
        mass = mass.reshape(-1)
    h64 = torch.from_numpy(np.ascontiguousarray(state[[m for _, m in hi]]).reshape(len(hi), state.shape[1]))
    h = h64.to(sl.hi_dtype(plan.tier))
    assert torch.equal(h.to(torch.float64), h64), "state not representable in the tier"
    return mass.contiguous(), h.cuda().contiguous()


def download_nd(mass, hi, plan):
    import torch
    pm = plan.plane_map()
    m = mass.detach().to("cpu", torch.float64).numpy().reshape(plan.n_lo, plan.cells)
    h = hi.detach().to("cpu").to(torch.float64).numpy().reshape(plan.n_hi, plan.cells)
    out = np.empty((plan.modes, plan.cells))
    for mode, v in enumerate(pm):
        out[mode] = m[-1 - v] if v < 0 else h[v]
    return out


def assert_sweep_close(got, want, mag, tier, k, what="", keep=None):
    tol = sweep_bound(want, got, mag, tier, k, keep)
    err = np.abs(got - want)
    bad = err > tol
    if np.any(bad):
        idx = np.argwhere(bad)[:5]
        msg = ", ".join(f"(m={m}, c={c}): got {got[m, c]!r} want {want[m, c]!r} tol {tol[m, c]:.3g}"
                        for m, c in idx)
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} elements out of bound: {msg}")
    # fraction of the rounded (non-FP64) coefficients that are not bit-identical
    if keep is None:
        return float(np.mean(got[1:] != want[1:]))
    rk = ~np.asarray(keep, dtype=bool)
    return float(np.mean(got[rk] != want[rk])) if rk.any() else 0.0


def weighted_rel_l2(got, want, ndim, k):
    from oracle import sldg_oracle as O
    w = O.mode_weights(ndim, k)[:, None]
    num = math.sqrt(float(np.sum(w * (got - want) ** 2)))
    den = math.sqrt(float(np.sum(w * want ** 2)))
    return num / den
