"""Plain, slow, obviously correct CPU FP64 oracle of the sLdG projection sweep.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code, header, table or
constant generator with the HIP library; the two meet only through data
(seeded inputs, which the tests hand to both sides).

Method (L. Einkemmer, "A mixed precision semi-Lagrangian algorithm and its
performance on accelerators", arXiv 1603.07008):

* Section II, eq. (1): Cheng-Knorr splitting reduces the Vlasov equation to 1D
  constant-coefficient advections u_t + a u_x = 0, each solved exactly along
  characteristics followed by an L2 projection (section II-A).
* Section II-A: in each cell the solution is a polynomial of degree k written
  in the Legendre basis, u = sum_j c_j P_j(2(x - x_i)/h); the coefficients
  follow eq. (cj), c_j = (2j+1)/2 * int_{-1}^{1} u P_j.
* Section II-A, update rule: the projection of the translated approximant gives
  c_new[i] = A c[i-s] + B c[i-s-1], with A, B in R^{o x o}, o = k+1, depending
  only on the fractional part of the displacement.
* Section II-A (storage of c_0) and section III-A: c_0, the cell mean, is kept
  in double precision and the higher modes in a narrower format, which keeps
  the mass conserved to double precision.

Readings of the paper taken here (each one is listed in the design notes):
* The displacement sigma = a*dt/h is in cells; s = floor(sigma) (the integer
  part of the CFL number in section II-A, read as floor so that the fractional
  part alpha lies in [0, 1) for either sign), then alpha is snapped so that
  alpha + (1 - alpha) == 1 exactly in FP64; an alpha that rounds to 1 is taken
  as s + 1, alpha = 0.
* A and B are the exact values of their defining integrals, evaluated here in
  exact rational arithmetic and rounded once to FP64 (the paper notes that
  Gauss-Legendre quadrature evaluates them exactly; rational arithmetic gives
  the same numbers without the quadrature's rounding).
* The grid is periodic in every dimension; in several dimensions each line
  (fixed transverse cell) uses the displacement at its transverse cell centre.
* Mass = (prod h) * sum of c_0 (c_0 is the cell mean).
"""
import ctypes
import math
import os
from fractions import Fraction

import numpy as np

from . import build as _build

TIERS = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3}

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        lib.oracle_sweep.restype = None
        lib.oracle_sweep.argtypes = [
            ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        lib.oracle_sweep_adjoint.restype = None
        lib.oracle_sweep_adjoint.argtypes = [
            ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_round_tier.restype = ctypes.c_double
        lib.oracle_round_tier.argtypes = [ctypes.c_double, ctypes.c_int]
        lib.oracle_round_array.restype = None
        lib.oracle_round_array.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        lib.oracle_set_threads.restype = None
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def num_threads():
    """OpenMP threads the oracle's C sweep runs on."""
    return _load().oracle_num_threads()


def set_threads(n):
    """Sets the OpenMP threads of later C sweeps (for timing the oracle)."""
    _load().oracle_set_threads(int(n))


# ---------------------------------------------------------------------------
# Legendre polynomials and the projection matrices (section II-A)
# ---------------------------------------------------------------------------

def legendre_monomial(j):
    """Exact monomial coefficients (ascending powers) of P_j on [-1, 1].

    Bonnet's recurrence (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}, P_0 = 1,
    P_1 = x (the Legendre polynomials of section II-A)."""
    prev, cur = [Fraction(1)], [Fraction(0), Fraction(1)]
    if j == 0:
        return prev
    for nn in range(1, j):
        xcur = [Fraction(0)] + cur
        prevp = prev + [Fraction(0)] * (len(xcur) - len(prev))
        nxt = [(Fraction(2 * nn + 1) * a - Fraction(nn) * b) / (nn + 1)
               for a, b in zip(xcur, prevp)]
        prev, cur = cur, nxt
    return cur


def _poly_shift(p, c):
    """Coefficients of q(x) = p(x - c) (binomial expansion)."""
    out = [Fraction(0)] * len(p)
    for m, a in enumerate(p):
        if a == 0:
            continue
        for r in range(m + 1):
            out[r] += a * math.comb(m, r) * (-c) ** (m - r)
    return out


def _poly_mul(p, q):
    out = [Fraction(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def _poly_integral(p, a, b):
    """int_a^b p(x) dx, exactly."""
    tot = Fraction(0)
    for m, c in enumerate(p):
        tot += c * (b ** (m + 1) - a ** (m + 1)) / (m + 1)
    return tot


def snap_shift(sigma):
    """Displacement in cells -> (s, alpha), alpha in [0, 1), alpha + (1-alpha) == 1.

    s is the integer part of the displacement (section II-A, update rule),
    read as floor."""
    sigma = float(sigma)
    s = math.floor(sigma)
    alpha = sigma - s
    beta = 1.0 - alpha
    alpha = 1.0 - beta
    if alpha >= 1.0:          # sigma just below an integer rounded up
        s, alpha = s + 1, 0.0
    return int(s), float(alpha)


def ab_exact(alpha, k):
    """A(alpha), B(alpha) of section II-A's update rule, correctly rounded to FP64.

    For cell i and displacement s + alpha (cells), the translated approximant
    restricted to cell i comes from cell i-s on xi in [2 alpha - 1, 1] (local
    coordinate xi - 2 alpha there) and from cell i-s-1 on xi in [-1, 2 alpha - 1]
    (local coordinate xi - 2 alpha + 2).  Projecting with eq. (cj):
        A[j][l] = (2j+1)/2 int_{2a-1}^{1}  P_j(xi) P_l(xi - 2a) dxi
        B[j][l] = (2j+1)/2 int_{-1}^{2a-1} P_j(xi) P_l(xi - 2a + 2) dxi
    The integrands are polynomials, so the integrals are evaluated exactly in
    rational arithmetic and rounded once."""
    a = Fraction(alpha)
    o = k + 1
    P = [legendre_monomial(j) for j in range(o)]
    A = np.zeros((o, o))
    B = np.zeros((o, o))
    for l in range(o):
        pa = _poly_shift(P[l], 2 * a)
        pb = _poly_shift(P[l], 2 * a - 2)
        for j in range(o):
            w = Fraction(2 * j + 1, 2)
            A[j, l] = float(w * _poly_integral(_poly_mul(P[j], pa), 2 * a - 1, Fraction(1)))
            B[j, l] = float(w * _poly_integral(_poly_mul(P[j], pb), Fraction(-1), 2 * a - 1))
    return A, B


_ab_cache = {}


def line_tables(sigma, k):
    """Per-line (s, [A; B]) tables for an array of displacements (cells)."""
    sigma = np.ascontiguousarray(sigma, dtype=np.float64).ravel()
    o = k + 1
    s_tab = np.empty(sigma.size, dtype=np.int32)
    ab_tab = np.empty((sigma.size, 2, o, o), dtype=np.float64)
    for t, sg in enumerate(sigma):
        s, alpha = snap_shift(sg)
        key = (alpha, k)
        if key not in _ab_cache:
            _ab_cache[key] = ab_exact(alpha, k)
        A, B = _ab_cache[key]
        s_tab[t] = s
        ab_tab[t, 0] = A
        ab_tab[t, 1] = B
    return s_tab, ab_tab


# ---------------------------------------------------------------------------
# Grid helpers
# ---------------------------------------------------------------------------

def n_modes(ndim, k):
    return (k + 1) ** ndim


def n_cells(ns):
    return int(np.prod(ns))


def line_strides(ns, dep):
    """Stride of each dimension in a per-line table indexed over the dims in
    `dep` (dimension 0 fastest), 0 for the other dimensions."""
    st = np.zeros(len(ns), dtype=np.int64)
    acc = 1
    for e in sorted(dep):
        st[e] = acc
        acc *= ns[e]
    return st, acc


# ---------------------------------------------------------------------------
# Sweep (section II-A update rule), via the plain C loops in sweep.c
# ---------------------------------------------------------------------------

def fp64_modes(ndim, k, ndouble=1):
    """Modes kept in FP64: total degree j_0 + ... + j_{d-1} below ndouble (the
    leading coefficients, c_j ~ h^|j| for smooth data, section II-A)."""
    o = k + 1
    keep = np.zeros(o ** ndim, dtype=np.uint8)
    for m in range(o ** ndim):
        deg = sum((m // o ** e) % o for e in range(ndim))
        keep[m] = 1 if deg < ndouble else 0
    return keep


def _scale_array(scale, M):
    if scale is None:
        return None
    e = np.ascontiguousarray(scale, dtype=np.int32).ravel()
    if e.size != M:
        raise ValueError(f"need {M} storage exponents, got {e.size}")
    return e


def sweep(state, ns, k, dim, sigma, dep=(), tier="fp64", sel=None, absolute=False, ndouble=1,
          scale=None):
    """One sLdG projection sweep along `dim`.

    state  float64 [o^ndim, cells] (mode-major, cells dimension-0 fastest)
    sigma  displacement in cells per line, indexed over the dims in `dep`
           (dimension 0 fastest); a scalar when dep is empty
    tier   storage emulation for modes m != 0 ('fp64', 'fp32', 'bf16', 'fp16')
    sel    optional int64 array of output cells; then the result is
           [o^ndim, len(sel)]
    ndouble number of leading modes kept in FP64 (fp64_modes)
    scale  optional int [o^ndim]: narrow mode m is stored as c * 2^scale[m],
           so its emulated value is round(c * 2^e) * 2^-e
    absolute  use |A|, |B| and |state| (no rounding): gives the magnitude
           sum_l |A_jl x_l| + |B_jl y_l| of every output, which bounds the
           rounding error of any evaluation order of the update
    """
    ns = [int(v) for v in ns]
    ndim = len(ns)
    if dim in dep:
        raise ValueError("the displacement of a sweep cannot depend on the swept dimension")
    state = np.ascontiguousarray(state, dtype=np.float64)
    M, C = n_modes(ndim, k), n_cells(ns)
    if state.shape != (M, C):
        raise ValueError(f"state shape {state.shape} != {(M, C)}")
    stride, ntab = line_strides(ns, dep)
    sigma = np.atleast_1d(np.asarray(sigma, dtype=np.float64)).ravel()
    if sigma.size != ntab:
        raise ValueError(f"need {ntab} displacements, got {sigma.size}")
    s_tab, ab_tab = line_tables(sigma, k)
    if absolute:
        ab_tab = np.abs(ab_tab)
        state = np.abs(state)
        tier = "fp64"
    if sel is None:
        out = np.empty((M, C))
        nsel, selp = C, None
    else:
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        out = np.empty((M, sel.size))
        nsel, selp = sel.size, sel.ctypes.data
    nsarr = np.asarray(ns, dtype=np.int64)
    keep = fp64_modes(ndim, k, ndouble)
    sc = _scale_array(scale, M)
    _load().oracle_sweep(ndim, nsarr.ctypes.data, k, dim, stride.ctypes.data,
                         s_tab.ctypes.data, ab_tab.ctypes.data, TIERS[tier], keep.ctypes.data,
                         None if sc is None else sc.ctypes.data,
                         state.ctypes.data, out.ctypes.data, nsel, selp)
    return out


def sweep_adjoint(grad, ns, k, dim, sigma, dep=(), absolute=False):
    """Transpose of `sweep` (FP64, no rounding) with the same displacements:
    the gradient with respect to the sweep's input of a function of its
    output, given the gradient with respect to the output.  With `absolute`,
    |A|, |B| and |grad|: the magnitude sum of every output, which bounds the
    rounding error of any evaluation order (as in `sweep`)."""
    ns = [int(v) for v in ns]
    ndim = len(ns)
    if dim in dep:
        raise ValueError("the displacement of a sweep cannot depend on the swept dimension")
    grad = np.ascontiguousarray(grad, dtype=np.float64)
    M, C = n_modes(ndim, k), n_cells(ns)
    if grad.shape != (M, C):
        raise ValueError(f"gradient shape {grad.shape} != {(M, C)}")
    stride, ntab = line_strides(ns, dep)
    sigma = np.atleast_1d(np.asarray(sigma, dtype=np.float64)).ravel()
    if sigma.size != ntab:
        raise ValueError(f"need {ntab} displacements, got {sigma.size}")
    s_tab, ab_tab = line_tables(sigma, k)
    if absolute:
        ab_tab = np.abs(ab_tab)
        grad = np.abs(grad)
    out = np.empty((M, C))
    nsarr = np.asarray(ns, dtype=np.int64)
    _load().oracle_sweep_adjoint(ndim, nsarr.ctypes.data, k, dim, stride.ctypes.data,
                                 s_tab.ctypes.data, ab_tab.ctypes.data, grad.ctypes.data,
                                 out.ctypes.data)
    return out


def run_sequence_adjoint(grad, ns, k, seq, steps=1):
    """Transpose of run_sequence (FP64): the sweeps' adjoints in reverse order."""
    for _ in range(steps):
        for dim, sigma, dep in reversed(seq):
            grad = sweep_adjoint(grad, ns, k, dim, sigma, dep)
    return grad


def round_tier(x, tier):
    """Round-to-nearest-even of every element onto the tier's storage format."""
    x = np.array(x, dtype=np.float64, copy=True)
    _load().oracle_round_array(x.ctypes.data, x.size, TIERS[tier])
    return x


def to_tier(state, tier, ndouble=1, k=None, ndim=None, scale=None):
    """Emulated storage of a state: the FP64 modes (by default mode 0 alone)
    stay, the others are rounded (scaled by 2^scale[m] first and back after,
    when storage exponents are given).  k and ndim are needed when
    ndouble != 1."""
    out = np.array(state, dtype=np.float64, copy=True)
    if tier != "fp64" and scale is not None:
        e = _scale_array(scale, out.shape[0])
        keep = np.zeros(out.shape[0], dtype=bool)
        if ndouble == 1:
            keep[0] = True
        else:
            if k is None or ndim is None:
                raise ValueError("to_tier needs k and ndim when ndouble != 1")
            keep = fp64_modes(ndim, k, ndouble).astype(bool)
        for m in np.nonzero(~keep)[0]:
            out[m] = np.ldexp(round_tier(np.ldexp(out[m], int(e[m])), tier), -int(e[m]))
    elif tier != "fp64":
        if ndouble == 1:
            keep = np.zeros(out.shape[0], dtype=bool)
            keep[0] = True
        else:
            if k is None or ndim is None:
                raise ValueError("to_tier needs k and ndim when ndouble != 1")
            keep = fp64_modes(ndim, k, ndouble).astype(bool)
        out[~keep] = round_tier(out[~keep], tier)
    return out


def run_sequence(state, ns, k, seq, tier="fp64", steps=1, ndouble=1, scale=None):
    """Apply a list of sweeps (dim, sigma, dep) `steps` times (section II,
    eq. (1): the split step is a composition of 1D advections)."""
    for _ in range(steps):
        for dim, sigma, dep in seq:
            state = sweep(state, ns, k, dim, sigma, dep, tier, ndouble=ndouble, scale=scale)
    return state


# ---------------------------------------------------------------------------
# FP16 storage with per-mode power-of-two scaling
#
# FP16 keeps 11 significant bits but only the exponents -14..15 in its normal
# range, so the small higher Legendre modes (c_j ~ h^|j| for smooth data,
# section II-A) fall into its subnormal range or flush to zero.  A narrow
# mode m is therefore stored as c * 2^e[m]; e[m] is chosen from the mode's
# absolute maximum `amax[m]` so that the stored values sit a fixed number of
# binades (the headroom) below 2^15.  A sweep predicts the exponents of its
# outputs from the absmax of its inputs (same mode), records the absmax of
# what it computes, and a mode whose values reach 2^15 at the predicted
# exponent (growth beyond the headroom in one sweep) is stored again at the
# exponent of its own absmax.  The absmax is kept rounded to FP32.
# ---------------------------------------------------------------------------

FP16_TOP = 15                 # 2^15 <= 65504 (largest finite FP16) < 2^16
SCALE_HEADROOM = 8            # binades kept free above a mode's absmax
SCALE_REPAIR_HEADROOM = 1     # headroom of a mode stored again after growth
SCALE_EMIN, SCALE_EMAX = -100, 100


def storage_exponent(amax, headroom):
    """The exponent e with 2^(14 - headroom) <= amax * 2^e < 2^(15 - headroom)
    (clamped to [-100, 100]); None when amax is 0 or not finite."""
    amax = float(amax)
    if not (amax > 0.0 and math.isfinite(amax)):
        return None
    _, x = math.frexp(amax)              # amax = f 2^x, 0.5 <= f < 1
    return min(max(FP16_TOP - headroom - x, SCALE_EMIN), SCALE_EMAX)


def _f32(x):
    return float(np.float32(x))


def to_scaled(state, k, ndim, ndouble=1, headroom=SCALE_HEADROOM):
    """FP16 storage of an FP64 state with per-mode scaling.  Returns
    (values, exps, amax): the values the stored numbers represent, the
    storage exponent of every mode (0 for the FP64 modes) and every narrow
    mode's absmax, rounded to FP32."""
    state = np.asarray(state, dtype=np.float64)
    keep = fp64_modes(ndim, k, ndouble).astype(bool)
    M = state.shape[0]
    e = np.zeros(M, dtype=np.int32)
    amax = np.zeros(M)
    for m in range(M):
        if keep[m] or state.shape[1] == 0:
            continue
        amax[m] = _f32(np.max(np.abs(state[m])))
        em = storage_exponent(amax[m], headroom)
        e[m] = 0 if em is None else em
    return to_tier(state, "fp16", ndouble, k, ndim, scale=e), e, amax


def sweep_scaled(state, exps, amax, ns, k, dim, sigma, dep=(), ndouble=1,
                 headroom=SCALE_HEADROOM):
    """One sweep of a scaled FP16 state (values, exps, amax as to_scaled
    returns them); returns the output in the same form."""
    ndim = len(ns)
    keep = fp64_modes(ndim, k, ndouble).astype(bool)
    acc = sweep(state, ns, k, dim, sigma, dep, "fp64")      # the update, unrounded
    M = acc.shape[0]
    e_out = np.array(exps, dtype=np.int32, copy=True)
    a_out = np.zeros(M)
    for m in range(M):
        if keep[m]:
            continue
        pred = storage_exponent(amax[m], headroom)
        if pred is None:
            pred = int(exps[m])
        a = _f32(np.max(np.abs(acc[m]))) if acc.shape[1] else 0.0
        a_out[m] = a
        if math.isfinite(a) and math.ldexp(a, pred) >= 2.0 ** FP16_TOP:
            pred = storage_exponent(a, SCALE_REPAIR_HEADROOM)
        e_out[m] = pred
    return to_tier(acc, "fp16", ndouble, k, ndim, scale=e_out), e_out, a_out


def run_sequence_scaled(scaled, ns, k, seq, steps=1, ndouble=1, headroom=SCALE_HEADROOM):
    """run_sequence for a scaled FP16 state (values, exps, amax)."""
    st, e, a = scaled
    for _ in range(steps):
        for dim, sigma, dep in seq:
            st, e, a = sweep_scaled(st, e, a, ns, k, dim, sigma, dep, ndouble, headroom)
    return st, e, a


# ---------------------------------------------------------------------------
# Transverse Gauss-node collocation
#
# With the displacement of a sweep along d depending on a transverse
# coordinate y (dimension t), the cell-centre sweep gives every line of a
# transverse cell the displacement at the cell centre (section II-A applied
# line by line).  The collocated sweep instead takes the state at the o
# Gauss-Legendre nodes y_q of the transverse cell (modal -> nodal in j_t),
# sweeps each node line with its own displacement sigma(y_q) (the update rule
# of section II-A, unchanged), and projects back onto the Legendre modes in
# y with the Gauss weights (nodal -> modal, eq. (cj) with the o-point rule).
# ---------------------------------------------------------------------------

def sweep_collocated(state, ns, k, dim, tdim, node_sigma, tier="fp64", ndouble=1):
    """One collocated sweep along `dim`, nodes in `tdim`.
    node_sigma: displacement in cells [N_tdim, o] (transverse cell, node)."""
    ns = [int(v) for v in ns]
    ndim = len(ns)
    o = k + 1
    if dim == tdim:
        raise ValueError("the transverse dimension must differ from the swept one")
    sig = np.asarray(node_sigma, dtype=np.float64).reshape(ns[tdim], o)
    st = np.asarray(state, dtype=np.float64)
    shape = [o] * ndim + ns[::-1]
    X = st.reshape(shape)
    jax = lambda e: ndim - 1 - e              # mode axis of dimension e
    iax = lambda e: 2 * ndim - 1 - e          # cell axis of dimension e
    xi, w = gauss_legendre(o)
    P = legendre_values(k, xi)                # [j, q]
    out = np.zeros_like(X)
    N = ns[dim]
    for q in range(o):
        nod = np.tensordot(P[:, q], X, axes=([0], [jax(tdim)]))        # j_t removed
        # axes of nod: modes without t (in order), then the cells
        jd = jax(dim) - (1 if jax(tdim) < jax(dim) else 0)
        it, idd = iax(tdim) - 1, iax(dim) - 1
        Y = np.moveaxis(nod, (jd, it, idd), (0, 1, -1))             # [j_d, N_t, ..., N_d]
        Z = np.empty_like(Y)
        s_tab, ab_tab = line_tables(sig[:, q], k)
        for i_t in range(ns[tdim]):
            s = int(s_tab[i_t])
            A, B = ab_tab[i_t, 0], ab_tab[i_t, 1]
            src = np.arange(N)
            ya = Y[:, i_t][..., (src - s) % N]
            yb = Y[:, i_t][..., (src - s - 1) % N]
            Z[:, i_t] = np.tensordot(A, ya, axes=([1], [0])) + np.tensordot(B, yb, axes=([1], [0]))
        back = np.moveaxis(Z, (0, 1, -1), (jd, it, idd))
        for jt in range(o):
            sl = [slice(None)] * (2 * ndim)
            sl[jax(tdim)] = jt
            out[tuple(sl)] += 0.5 * (2 * jt + 1) * w[q] * P[jt, q] * back
    res = out.reshape(st.shape)
    return to_tier(res, tier, ndouble, k, ndim) if tier != "fp64" else res


# ---------------------------------------------------------------------------
# Self-consistent field of a 1D-1V problem (x = dimension 0, v = dimension 1)
#
# The paper states the Vlasov equation with a given field E(x) (section II) and
# no field equation.  Reading taken: Gauss's law of the normalised
# Vlasov-Poisson system with a neutralising background, in the paper's sign
# convention (+E d_v f): dE/dx = rho - mean(rho), E periodic with zero mean,
# rho(x) = int f dv.  The v-sweep displacement of the line through x cell i is
# E at the cell centre times dt / h_v (lines use their transverse cell centre).
# ---------------------------------------------------------------------------

def density_moments(state, ns, k, hv):
    """rho in x cell i as a Legendre expansion: r[j, i] = h_v sum_iv c(i, iv;
    mode (j, 0)) (only the j_v = 0 modes integrate to non-zero over a v cell)."""
    nx, nv = ns
    o = k + 1
    st = np.asarray(state, dtype=np.float64)
    r = np.empty((o, nx))
    for j in range(o):
        plane = st[j].reshape(nv, nx)                  # cell = i_x + nx * i_v
        for i in range(nx):
            r[j, i] = hv * math.fsum(plane[:, i].tolist())
    return r


def _half_cell_left_integral(j):
    """int_{-1}^{0} P_j(xi) d xi, exactly."""
    p = legendre_monomial(j)
    acc = Fraction(0)
    for e, c in enumerate(p):
        acc += c * (Fraction(0) - Fraction((-1) ** (e + 1), e + 1))
    return acc


def poisson_field(state, ns, k, hx, hv):
    """E at the x cell centres, from dE/dx = rho - mean(rho), zero mean.
    Steps: the density moments; the mean density; the face values of the
    antiderivative of rho - mean(rho) (starting at 0); the cell means of that
    antiderivative; the constant that makes the mean zero; the centre values."""
    nx = ns[0]
    r = density_moments(state, ns, k, hv)
    rbar = math.fsum(r[0].tolist()) / nx
    faces = np.empty(nx + 1)
    faces[0] = 0.0
    for i in range(nx):
        faces[i + 1] = faces[i] + hx * (r[0, i] - rbar)
    # cell mean of the antiderivative: (1/h) int_cell F = F_i + h/2 (r0 - rbar) - h/6 r1
    means = [faces[i] + 0.5 * hx * (r[0, i] - rbar) - (hx / 6.0 * r[1, i] if k >= 1 else 0.0)
             for i in range(nx)]
    C = -math.fsum(means) / nx
    half = [float(_half_cell_left_integral(j)) for j in range(k + 1)]
    out = np.empty(nx)
    for i in range(nx):
        g = (r[0, i] - rbar) * half[0] + math.fsum(r[j, i] * half[j] for j in range(1, k + 1))
        out[i] = faces[i] + C + 0.5 * hx * g
    return out


def poisson_shift(state, ns, k, hx, hv, dt):
    """The v-sweep displacement (cells) per x line: E(x_i) dt / h_v."""
    return poisson_field(state, ns, k, hx, hv) * dt / hv


# ---------------------------------------------------------------------------
# Self-consistent field of (x1, x2, v1, v2) problems (section II: the Vlasov
# equation with E(x)).  Gauss's law div E = rho - mean(rho) with a curl-free
# periodic E = -grad phi, solved spectrally on the cell means of the density
# (the c_0 of the x cells): the cell means are divided by the Fourier symbol of
# cell averaging, sinc(kappa_1 h_1/2) sinc(kappa_2 h_2/2), so the solve is
# exact for densities that are trigonometric polynomials resolved by the grid;
# the Nyquist modes and the mean are dropped.  E at the x cell centres; the
# v1 (v2) sweep of the line through x cell (i1, i2) moves by E_1 dt / h_v1
# (E_2 dt / h_v2).
# ---------------------------------------------------------------------------

def density_means_2d(state, ns, hv1, hv2):
    """Cell means of rho(x1, x2) = int int f dv1 dv2 over the x cells:
    h_v1 h_v2 times the sum over the v cells of c_0 (the mean of f over a v
    cell integrates to h_v1 h_v2 c_0).  Shape [N2, N1] (x1 fastest)."""
    n1, n2, m1, m2 = ns
    c0 = np.asarray(state[0], dtype=np.float64).reshape(m2, m1, n2, n1)
    out = np.empty((n2, n1))
    for i2 in range(n2):
        for i1 in range(n1):
            out[i2, i1] = hv1 * hv2 * math.fsum(c0[:, :, i2, i1].ravel().tolist())
    return out


def _wavenumbers(n, h):
    """Angular wave numbers 2 pi m / (n h) of the DFT indices 0..n-1 (m taken
    in (-n/2, n/2]), and whether each is the Nyquist index of an even n."""
    m = np.array([j if j <= n // 2 else j - n for j in range(n)], dtype=np.float64)
    nyq = np.array([n % 2 == 0 and j == n // 2 for j in range(n)])
    return 2.0 * math.pi * m / (n * h), nyq


def poisson_field_2d(state, ns, h):
    """(E_1, E_2) at the x cell centres, each flattened with x1 fastest.
    h = (h_x1, h_x2, h_v1, h_v2).  Steps: the cell means of rho; their 2D DFT
    (library FFT); per wave vector kappa != 0 without a Nyquist index, the
    point-value Fourier coefficient rho_hat / (sinc(kappa_1 h_1/2)
    sinc(kappa_2 h_2/2)) and E_hat = -i kappa rho_hat / |kappa|^2 (from
    -lap phi = rho - mean, E = -grad phi); the inverse DFT at the centres."""
    n1, n2 = ns[0], ns[1]
    rho = density_means_2d(state, ns, h[2], h[3])
    R = np.fft.fft2(rho)                              # axis 0: x2, axis 1: x1
    k1, nyq1 = _wavenumbers(n1, h[0])
    k2, nyq2 = _wavenumbers(n2, h[1])
    E1h = np.zeros((n2, n1), dtype=complex)
    E2h = np.zeros((n2, n1), dtype=complex)
    for a in range(n2):
        for b in range(n1):
            if nyq1[b] or nyq2[a] or (k1[b] == 0.0 and k2[a] == 0.0):
                continue
            s1 = math.sin(0.5 * k1[b] * h[0]) / (0.5 * k1[b] * h[0]) if k1[b] != 0.0 else 1.0
            s2 = math.sin(0.5 * k2[a] * h[1]) / (0.5 * k2[a] * h[1]) if k2[a] != 0.0 else 1.0
            rho_pt = R[a, b] / (s1 * s2)
            kk = k1[b] ** 2 + k2[a] ** 2
            E1h[a, b] = -1j * k1[b] * rho_pt / kk
            E2h[a, b] = -1j * k2[a] * rho_pt / kk
    E1 = np.real(np.fft.ifft2(E1h))
    E2 = np.real(np.fft.ifft2(E2h))
    return E1.ravel(), E2.ravel()


def poisson_shift_2d(state, ns, h, dt):
    """The v1- and v2-sweep displacements (cells) per x line (x1 fastest):
    E_1 dt / h_v1 and E_2 dt / h_v2."""
    E1, E2 = poisson_field_2d(state, ns, h)
    return E1 * dt / h[2], E2 * dt / h[3]


# ---------------------------------------------------------------------------
# Initial projection, eq. (cj)
# ---------------------------------------------------------------------------

def gauss_legendre(nq):
    """Gauss-Legendre nodes and weights on [-1, 1] (library routine)."""
    return np.polynomial.legendre.leggauss(nq)


def legendre_values(k, xi):
    """P_0..P_k at points xi (Bonnet's recurrence in FP64), shape [k+1, len(xi)]."""
    xi = np.asarray(xi, dtype=np.float64)
    out = np.zeros((k + 1,) + xi.shape)
    out[0] = 1.0
    if k >= 1:
        out[1] = xi
    for nn in range(1, k):
        out[nn + 1] = ((2 * nn + 1) * xi * out[nn] - nn * out[nn - 1]) / (nn + 1)
    return out


def project_1d(f, n, lo, hi, k, nq=None):
    """Eq. (cj) on a 1D grid with an nq-point Gauss-Legendre rule (default k+1).
    Returns [k+1, n]."""
    nq = k + 1 if nq is None else nq
    xg, wg = gauss_legendre(nq)
    h = (hi - lo) / n
    centres = lo + (np.arange(n) + 0.5) * h
    x = centres[None, :] + 0.5 * h * xg[:, None]              # [nq, n]
    fx = np.asarray(f(x), dtype=np.float64)
    P = legendre_values(k, xg)                                 # [o, nq]
    coef = np.empty((k + 1, n))
    for j in range(k + 1):
        coef[j] = (2 * j + 1) / 2.0 * np.sum(wg[:, None] * P[j][:, None] * fx, axis=0)
    return coef


def project_separable(terms, ns, los, his, k, nq=None):
    """Eq. (cj) in several dimensions for f = sum_t prod_e f_{t,e}(x_e).

    A tensor Gauss rule applied to a product function factorises, so the
    tensor-product coefficients are the outer product of the 1D ones."""
    ndim = len(ns)
    M, C = n_modes(ndim, k), n_cells(ns)
    out = np.zeros((M, C))
    for term in terms:
        c1 = [project_1d(term[e], ns[e], los[e], his[e], k, nq) for e in range(ndim)]
        # mode index j_0 fastest, cell index i_0 fastest -> build with reversed axes
        t = c1[ndim - 1]
        for e in range(ndim - 2, -1, -1):
            # t: [o^(ndim-1-e), cells_hi]; prepend dim e as the faster index
            t = (t[:, None, :, None] * c1[e][None, :, None, :]).reshape(
                t.shape[0] * (k + 1), t.shape[1] * ns[e])
        out += t
    return out


# ---------------------------------------------------------------------------
# Diagnostics
# ---------------------------------------------------------------------------

def cell_volume(ns, los, his):
    return float(np.prod([(his[e] - los[e]) / ns[e] for e in range(len(ns))]))


def mass(state, ns, los, his):
    """Total mass = (prod h) * sum of the cell means c_0 (section II-A: c_0 is
    the mass of the cell up to the factor h), summed exactly (math.fsum)."""
    return cell_volume(ns, los, his) * math.fsum(np.asarray(state[0], dtype=np.float64).tolist())


def mass_sum(mass_plane):
    """Exactly rounded sum of a mass array."""
    return math.fsum(np.asarray(mass_plane, dtype=np.float64).ravel().tolist())


def mode_weights(ndim, k):
    """Integral over a cell of (prod_e P_{j_e})^2 divided by the cell volume,
    prod_e 1/(2 j_e + 1), for every mode id m = j_0 + o*(j_1 + ...)."""
    o = k + 1
    w = np.ones(o ** ndim)
    for m in range(o ** ndim):
        for e in range(ndim):
            j = (m // o ** e) % o
            w[m] /= 2 * j + 1
    return w


def weighted_l2_sq(state, ns, los, his):
    """||u_h||_{L2}^2 = (prod h) * sum_cells sum_m c_m^2 prod_e 1/(2 j_e + 1)."""
    ndim = len(ns)
    k = round(state.shape[0] ** (1.0 / ndim)) - 1
    w = mode_weights(ndim, k)
    return cell_volume(ns, los, his) * float(np.sum(w[:, None] * np.asarray(state) ** 2))


def eval_1d(coef, n, lo, hi, x):
    """Evaluate a 1D piecewise Legendre expansion [k+1, n] at points x (periodic)."""
    k = coef.shape[0] - 1
    h = (hi - lo) / n
    y = (np.asarray(x, dtype=np.float64) - lo) / h
    i = np.floor(y).astype(np.int64)
    xi = 2.0 * (y - i) - 1.0
    i = np.mod(i, n)
    P = legendre_values(k, xi)
    return np.sum(coef[:, i] * P, axis=0)


def l2_error_1d(coef, n, lo, hi, f, nq=None):
    """||u_h - f||_{L2} on a 1D periodic grid with an nq-point Gauss rule per
    cell (default k+4)."""
    k = coef.shape[0] - 1
    nq = k + 4 if nq is None else nq
    xg, wg = gauss_legendre(nq)
    h = (hi - lo) / n
    centres = lo + (np.arange(n) + 0.5) * h
    x = centres[None, :] + 0.5 * h * xg[:, None]
    P = legendre_values(k, xg)                      # [o, nq]
    uh = np.einsum("jq,jn->qn", P, coef)
    err = uh - f(x)
    return math.sqrt(0.5 * h * float(np.sum(wg[:, None] * err ** 2)))
