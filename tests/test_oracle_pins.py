"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these compares the oracle with itself: each check uses an independent
computation (numerical quadrature of the defining integrals, a brute-force
projection, library rounding routines, closed forms) or an invariant of the
method (section II-A: exact translation + L2 projection, mass conservation,
locality, order k+1).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import sldg_oracle as O
from paper_1603_07008_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
rng0 = np.random.default_rng(20160323)


# --------------------------------------------------------------------------
# storage-format rounding (section II-A / III-A: higher modes in a narrower
# format, round to nearest even)
# --------------------------------------------------------------------------

def _sample_doubles(n, rng):
    mant = rng.uniform(-2, 2, n)
    expo = rng.integers(-160, 140, n)
    x = np.ldexp(mant, expo)
    return np.concatenate([x, [0.0, -0.0, 1.0, -1.5, 65504.0, 65520.0, 6e-8, 3e-8]])


def test_round_fp32_matches_numpy_cast():
    x = _sample_doubles(20000, rng0)
    x = x[np.abs(x) < 3e38]
    got = O.round_tier(x, "fp32")
    want = x.astype(np.float32).astype(np.float64)
    assert np.array_equal(got, want)


def test_round_fp16_matches_numpy_cast():
    x = _sample_doubles(20000, rng0)
    x = x[np.abs(x) < 1e6]
    with np.errstate(over="ignore"):
        want = x.astype(np.float16).astype(np.float64)
    got = O.round_tier(x, "fp16")
    assert np.array_equal(got, want)


def test_round_bf16_matches_torch_on_fp32_values_and_ties():
    torch = pytest.importorskip("torch")
    x = _sample_doubles(20000, rng0)
    x = x[np.abs(x) < 3e38].astype(np.float32).astype(np.float64)
    want = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = O.round_tier(x, "bf16")
    assert np.array_equal(got, want)
    # direct FP64 -> BF16 rounding, checked on hand-built cases: 1 + 2^-8 is the
    # midpoint between 1 and 1 + 2^-7 (ties to even -> 1), a hair above rounds up
    assert O.round_tier(np.array([1 + 2.0 ** -8]), "bf16")[0] == 1.0
    assert O.round_tier(np.array([1 + 2.0 ** -8 + 2.0 ** -40]), "bf16")[0] == 1 + 2.0 ** -7
    assert O.round_tier(np.array([1 + 3 * 2.0 ** -8]), "bf16")[0] == 1 + 2.0 ** -6


# --------------------------------------------------------------------------
# A(alpha), B(alpha) (section II-A, update rule)
# --------------------------------------------------------------------------

def _quad_ab(alpha, k, nq=12):
    """The defining integrals by numerical Gauss quadrature on each
    sub-interval (numpy's Legendre routines), independent of the oracle's
    rational arithmetic."""
    o = k + 1
    xg, wg = np.polynomial.legendre.leggauss(nq)
    A = np.zeros((o, o))
    B = np.zeros((o, o))
    e = [np.eye(o)[j] for j in range(o)]
    lv = np.polynomial.legendre.legval
    a, b = 2 * alpha - 1, 1.0
    xa = 0.5 * (b - a) * xg + 0.5 * (b + a)
    wa = 0.5 * (b - a) * wg
    a2, b2 = -1.0, 2 * alpha - 1
    xb = 0.5 * (b2 - a2) * xg + 0.5 * (b2 + a2)
    wb = 0.5 * (b2 - a2) * wg
    for j in range(o):
        for l in range(o):
            A[j, l] = (2 * j + 1) / 2 * np.sum(wa * lv(xa, e[j]) * lv(xa - 2 * alpha, e[l]))
            B[j, l] = (2 * j + 1) / 2 * np.sum(wb * lv(xb, e[j]) * lv(xb - 2 * alpha + 2, e[l]))
    return A, B


@pytest.mark.parametrize("k", [1, 2, 3])
def test_ab_matches_numerical_quadrature(k):
    for alpha in [0.0, 0.1, 0.37, 0.5, 0.77, 0.999, 1e-9]:
        A, B = O.ab_exact(alpha, k)
        Aq, Bq = _quad_ab(alpha, k)
        assert np.max(np.abs(A - Aq)) < 5e-15
        assert np.max(np.abs(B - Bq)) < 5e-15


def test_ab_hand_values_at_half():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "ab_k2_alpha_half.txt"))
            if ln.strip() and not ln.startswith("#")]
    A, B = O.ab_exact(0.5, 2)
    for name, j, l, val in rows:
        M = A if name == "A" else B
        assert M[int(j), int(l)] == float(Fraction(val)), (name, j, l)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_ab_limits_identity_and_shift(k):
    A, B = O.ab_exact(0.0, k)
    assert np.array_equal(A, np.eye(k + 1)) and np.array_equal(B, np.zeros((k + 1, k + 1)))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_ab_parity_symmetry(k):
    # reflecting x -> -x maps the problem with alpha to the one with 1 - alpha
    # and swaps the roles of the two source cells: B(a) = S A(1-a) S, S = diag((-1)^j)
    S = np.diag([(-1.0) ** j for j in range(k + 1)])
    for alpha in [0.125, 0.25, 0.375, 0.5, 0.8125]:      # exact complements
        A, B = O.ab_exact(alpha, k)
        A1, _ = O.ab_exact(1 - alpha, k)
        assert np.array_equal(B, S @ A1 @ S)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_ab_mass_row(k):
    # int P_l over a full cell vanishes for l >= 1 and is 2 for l = 0, so the
    # mass row satisfies A_00 + B_00 = 1 and A_0l + B_0l = 0 exactly
    for sigma in [0.37, -2.71, 5.999999999, 1e-17, -1e-17, 3.0]:
        s, alpha = O.snap_shift(sigma)
        assert 0.0 <= alpha < 1.0
        A, B = O.ab_exact(alpha, k)
        assert A[0, 0] + B[0, 0] == 1.0
        assert np.all(A[0, 1:] + B[0, 1:] == 0.0)


def test_snap_shift_floor_and_rounding_edge():
    assert O.snap_shift(0.37) == (0, 0.37)
    s, a = O.snap_shift(-0.25)
    assert (s, a) == (-1, 0.75)
    s, a = O.snap_shift(-1e-17)           # 1 - 1e-17 rounds to 1 -> next cell
    assert (s, a) == (0, 0.0)
    s, a = O.snap_shift(7.0)
    assert (s, a) == (7, 0.0)


# --------------------------------------------------------------------------
# the sweep against a brute-force projection (section II-A: translate exactly,
# then L2-project onto piecewise polynomials)
# --------------------------------------------------------------------------

def _brute_sweep_1d(coef, sigma, nq=None):
    """c'_ij = (2j+1)/2 int_{-1}^{1} u(x_i + xi h/2 - sigma h) P_j(xi) dxi,
    with u the piecewise Legendre expansion, integrated by Gauss quadrature on
    the two pieces between which the translated grid's cell boundary falls."""
    o, n = coef.shape
    k = o - 1
    nq = 2 * k + 2 if nq is None else nq
    xg, wg = np.polynomial.legendre.leggauss(nq)
    lv = np.polynomial.legendre.legval
    out = np.zeros_like(coef)
    frac = sigma - math.floor(sigma)
    cut = 2 * frac - 1                       # break point in local coordinates
    pieces = [(-1.0, cut), (cut, 1.0)] if 0 < frac else [(-1.0, 1.0)]
    for i in range(n):
        for a, b in pieces:
            if b <= a:
                continue
            xi = 0.5 * (b - a) * xg + 0.5 * (b + a)
            w = 0.5 * (b - a) * wg
            y = i + 0.5 + 0.5 * xi - sigma   # position in cell units
            src = np.floor(y).astype(int)
            loc = 2 * (y - src) - 1
            src = np.mod(src, n)
            u = np.array([lv(loc[q], coef[:, src[q]]) for q in range(len(xi))])
            for j in range(o):
                out[j, i] += (2 * j + 1) / 2 * np.sum(w * u * lv(xi, np.eye(o)[j]))
    return out


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("sigma", [0.37, -0.37, 2.6, -5.25, 0.999, 1e-3, 8.5])
def test_sweep_matches_bruteforce_1d(k, sigma):
    n = 7
    coef = rng0.standard_normal((k + 1, n))
    got = O.sweep(coef, (n,), k, 0, sigma)
    want = _brute_sweep_1d(coef, sigma)
    assert np.max(np.abs(got - want)) < 1e-13


def _brute_sweep_2d(state, ns, k, dim, sigma_lines):
    """Brute-force projection for a 2D tensor grid: apply the 1D brute force
    along `dim` for every transverse cell and every spectator mode."""
    o = k + 1
    n0, n1 = ns
    st = state.reshape(o, o, n1, n0)         # [j1, j0, i1, i0]
    out = np.zeros_like(st)
    if dim == 0:
        for i1 in range(n1):
            for j1 in range(o):
                out[j1, :, i1, :] = _brute_sweep_1d(st[j1, :, i1, :], sigma_lines[i1])
    else:
        for i0 in range(n0):
            for j0 in range(o):
                out[:, j0, :, i0] = _brute_sweep_1d(st[:, j0, :, i0], sigma_lines[i0])
    return out.reshape(o * o, n0 * n1)


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("dim", [0, 1])
def test_sweep_matches_bruteforce_2d(k, dim):
    ns = (5, 6)
    o = k + 1
    state = rng0.standard_normal((o * o, 30))
    other = 1 - dim
    sig = rng0.uniform(-3, 3, ns[other])
    got = O.sweep(state, ns, k, dim, sig, dep=(other,))
    want = _brute_sweep_2d(state, ns, k, dim, sig)
    assert np.max(np.abs(got - want)) < 1e-13


def test_sweep_3d_spectators_and_line_table_indexing():
    # a sweep along the middle dim of a 3D grid whose displacement depends on
    # dims 0 and 2 equals the 1D brute force on every line and spectator pair
    k, ns = 1, (3, 4, 5)
    o = k + 1
    state = rng0.standard_normal((o ** 3, 60))
    sig = rng0.uniform(-2, 2, 3 * 5)          # over (dim0, dim2), dim 0 fastest
    got = O.sweep(state, ns, k, 1, sig, dep=(0, 2))
    st = state.reshape(o, o, o, 5, 4, 3)      # [j2, j1, j0, i2, i1, i0]
    gt = got.reshape(o, o, o, 5, 4, 3)
    for i0 in range(3):
        for i2 in range(5):
            for j0 in range(o):
                for j2 in range(o):
                    w = _brute_sweep_1d(st[j2, :, j0, i2, :, i0], sig[i0 + 3 * i2])
                    assert np.max(np.abs(gt[j2, :, j0, i2, :, i0] - w)) < 1e-13


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("tier", ["fp64", "fp32", "bf16", "fp16"])
def test_integer_shift_is_exact_permutation(tier):
    k, ns = 2, (6, 5)
    o = k + 1
    state = O.to_tier(rng0.standard_normal((o * o, 30)), tier)
    sig = np.array([3.0, -1.0, 0.0, 7.0, -6.0])   # per line over dim 1
    got = O.sweep(state, ns, k, 0, sig, dep=(1,), tier=tier)
    st = state.reshape(o * o, 5, 6)
    want = np.empty_like(st)
    for i1 in range(5):
        want[:, i1, :] = np.roll(st[:, i1, :], int(sig[i1]), axis=1)
    assert np.array_equal(got, want.reshape(o * o, 30))


@pytest.mark.parametrize("tier", ["fp64", "fp32", "bf16", "fp16"])
def test_constants_preserved_bitwise(tier):
    k, ns = 3, (9, 4)
    o = k + 1
    state = np.zeros((o * o, 36))
    state[0] = 1.0
    sig = rng0.uniform(-4, 4, 9)
    got = O.sweep(state, ns, k, 1, sig, dep=(0,), tier=tier)
    assert np.array_equal(got, state)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_polynomials_of_degree_k_translate_exactly(k):
    # a global polynomial of degree <= k is in the approximation space, so its
    # translate is projected exactly; compare with numpy's monomial -> Legendre
    # conversion of the translated polynomial in every cell
    n, sigma = 12, 2.37
    h = 1.0 / n
    p = rng0.standard_normal(k + 1)             # monomial coefficients in x

    def cell_coeffs(shift):
        out = np.zeros((k + 1, n))
        P = np.polynomial.Polynomial(p)
        for i in range(n):
            xc = (i + 0.5) * h
            # q(xi) = p(xc + xi h/2 - shift), as a polynomial in xi
            q = P(np.polynomial.Polynomial([xc - shift, 0.5 * h]))
            out[:, i] = np.polynomial.legendre.poly2leg(q.coef)[: k + 1] if len(q.coef) >= k + 1 \
                else np.pad(np.polynomial.legendre.poly2leg(q.coef), (0, k + 1 - len(q.coef)))
        return out

    c0 = cell_coeffs(0.0)
    got = O.sweep(c0, (n,), k, 0, sigma)
    want = cell_coeffs(sigma * h)
    inner = np.arange(4, n)                      # sources not wrapped around
    assert np.max(np.abs(got[:, inner] - want[:, inner])) < 1e-12


def test_locality_two_cells():
    # output cell i depends only on cells i-s and i-s-1: perturbing one input
    # cell changes exactly two output cells (section II-A)
    k, n = 2, 16
    coef = rng0.standard_normal((k + 1, n))
    sigma = 3.4
    base = O.sweep(coef, (n,), k, 0, sigma)
    pert = coef.copy()
    pert[:, 5] += 1.0
    diff = np.any(O.sweep(pert, (n,), k, 0, sigma) != base, axis=0)
    assert sorted(np.nonzero(diff)[0].tolist()) == [8, 9]


@pytest.mark.parametrize("tier", ["fp64", "fp32", "bf16", "fp16"])
def test_mass_conserved_1d_oscillatory_long_run(tier):
    # section III-A: keeping c_0 in FP64 conserves mass to double precision;
    # an oscillatory initial value advected over 10^4 steps
    n, k, steps = 64, 2, 10000
    rng = np.random.default_rng(1603)
    m = np.arange(1, n // 4 + 1)
    r = rng.uniform(0, 1, m.size) / m
    ph = rng.uniform(0, 2 * np.pi, m.size)
    f = lambda x: 1.0 + np.sum(r[:, None, None] * np.sin(2 * np.pi * m[:, None, None] * x[None] + ph[:, None, None]), axis=0)
    c = O.to_tier(O.project_1d(f, n, 0.0, 1.0, k), tier)
    M0 = O.mass(c, (n,), (0.0,), (1.0,))
    scale = (1.0 / n) * math.fsum(np.abs(c[0]).tolist())
    for _ in range(steps):
        c = O.sweep(c, (n,), k, 0, 0.37, tier=tier)
    M1 = O.mass(c, (n,), (0.0,), (1.0,))
    assert abs(M1 - M0) / scale <= 1e-14


def test_weighted_l2_norm_never_grows():
    # the sweep is an L2 projection of an isometric translate, so the weighted
    # norm sum_m c_m^2 prod 1/(2j+1) cannot grow (up to rounding)
    p = inputs.vlasov_2d(nx=32, nv=32)
    c = O.project_separable(p.f0_terms, p.ns, p.los, p.his, p.k)
    eps = np.finfo(float).eps
    prev = O.weighted_l2_sq(c, p.ns, p.los, p.his)
    for _ in range(5):
        for sw in p.seq:
            c = O.sweep(c, p.ns, p.k, sw.dim, sw.sigma, sw.dep)
            cur = O.weighted_l2_sq(c, p.ns, p.los, p.his)
            assert cur <= prev * (1 + 8 * (p.k + 1) * eps)
            prev = cur
    # the plain (unweighted) coefficient norm is not the conserved quantity:
    # the weights matter for the statement above
    w = O.mode_weights(2, p.k)
    assert np.allclose(w[:3], [1, 1 / 3, 1 / 5]) and np.isclose(w[4], 1 / 9)


def test_weighted_l2_matches_quadrature_of_the_function():
    n, k = 10, 3
    coef = rng0.standard_normal((k + 1, n))
    xg, wg = np.polynomial.legendre.leggauss(8)
    h = 1.0 / n
    tot = 0.0
    for i in range(n):
        u = np.polynomial.legendre.legval(xg, coef[:, i])
        tot += 0.5 * h * np.sum(wg * u * u)
    assert math.isclose(O.weighted_l2_sq(coef, (n,), (0.0,), (1.0,)), tot, rel_tol=1e-13)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_order_of_convergence_k_plus_1(k):
    # section II-A: order o = k+1.  sin(2 pi x) advected exactly one period in
    # n = round(N/0.37) steps of sigma = N/n cells; the error halves by 2^(k+1)
    errs = []
    Ns = [16, 32, 64]
    for N in Ns:
        nsteps = round(N / 0.37)
        sigma = N / nsteps
        f = lambda x: np.sin(2 * np.pi * x)
        c = O.project_1d(f, N, 0.0, 1.0, k, nq=k + 4)
        for _ in range(nsteps):
            c = O.sweep(c, (N,), k, 0, sigma)
        errs.append(O.l2_error_1d(c, N, 0.0, 1.0, f))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(abs(r - (k + 1)) < 0.25 for r in rates), (errs, rates)


def test_literal_1d_config_against_exact_translate():
    p = inputs.advection_1d()
    f = p.f0_terms[0][0]
    c = O.project_1d(f, 64, 0.0, 1.0, p.k)
    for _ in range(p.steps):
        c = O.sweep(c, p.ns, p.k, 0, 0.37)
    T = 0.37 * p.steps / 64
    err = O.l2_error_1d(c, 64, 0.0, 1.0, lambda x: np.sin(2 * np.pi * (x - T)))
    # (k+1)-point Gauss initial projection + 270 projections at N = 64, k = 2
    assert err < 1e-5


# --------------------------------------------------------------------------
# initial projection, eq. (cj)
# --------------------------------------------------------------------------

def test_projection_of_polynomials_is_exact():
    k, n = 3, 5
    p = np.polynomial.Polynomial(rng0.standard_normal(k + 1))
    c = O.project_1d(p, n, -1.0, 2.0, k)
    x = np.linspace(-1.0, 2.0, 41)[1:-1]
    assert np.max(np.abs(O.eval_1d(c, n, -1.0, 2.0, x) - p(x))) < 1e-13


def test_separable_projection_equals_direct_tensor_rule():
    p = inputs.vlasov_2d(nx=6, nv=7)
    k, o = p.k, p.k + 1
    c = O.project_separable(p.f0_terms, p.ns, p.los, p.his, k)
    xg, wg = np.polynomial.legendre.leggauss(o)
    P = O.legendre_values(k, xg)
    f = lambda x, v: p.f0_terms[0][0](x) * p.f0_terms[0][1](v)
    hx, hv = p.h
    for i1 in range(7):
        for i0 in range(6):
            xc, vc = p.centres(0)[i0], p.centres(1)[i1]
            F = f(xc + 0.5 * hx * xg[:, None], vc + 0.5 * hv * xg[None, :])
            for j1 in range(o):
                for j0 in range(o):
                    want = (2 * j0 + 1) / 2 * (2 * j1 + 1) / 2 * np.sum(
                        wg[:, None] * wg[None, :] * P[j0][:, None] * P[j1][None, :] * F)
                    got = c[j0 + o * j1, i0 + 6 * i1]
                    assert abs(got - want) < 1e-15


# --------------------------------------------------------------------------
# adjoint (transpose) sweep
# --------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 2, 3])
def test_adjoint_dot_product_identity(k):
    # <M x, y> = <x, M^T y> for the sweep M and its oracle transpose
    rng = np.random.default_rng(50 + k)
    for ns, dim, dep in [((9,), 0, ()), ((7, 6), 1, (0,)), ((5, 4, 6), 0, (1, 2)),
                         ((4, 5, 3), 2, (0,))]:
        o = k + 1
        M, C = o ** len(ns), int(np.prod(ns))
        x = rng.standard_normal((M, C))
        y = rng.standard_normal((M, C))
        nsig = int(np.prod([ns[e] for e in dep])) if dep else 1
        sig = rng.uniform(-7, 7, nsig)
        lhs = math.fsum((O.sweep(x, ns, k, dim, sig, dep) * y).ravel().tolist())
        rhs = math.fsum((x * O.sweep_adjoint(y, ns, k, dim, sig, dep)).ravel().tolist())
        assert abs(lhs - rhs) <= 1e-13 * math.sqrt(M * C), (ns, dim, lhs, rhs)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_adjoint_equals_weighted_reflected_forward(k):
    # A(a)^T = W B(1-a) W^-1 and B(a)^T = W A(1-a) W^-1 with W = diag(2/(2j+1)):
    # so the transpose sweep is W F(-sigma) W^-1: the weight-conjugated forward
    # sweep with the opposite displacement (the projection is self-adjoint in
    # the L2 inner product, whose Gram matrix per cell is W)
    W = np.diag([2.0 / (2 * j + 1) for j in range(k + 1)])
    Wi = np.linalg.inv(W)
    for alpha in [0.125, 0.375, 0.5, 0.6875]:
        A, B = O.ab_exact(alpha, k)
        A1, B1 = O.ab_exact(1 - alpha, k)
        assert np.allclose(A.T, W @ B1 @ Wi, atol=1e-15, rtol=0)
        assert np.allclose(B.T, W @ A1 @ Wi, atol=1e-15, rtol=0)
    n = 11
    g = np.random.default_rng(5).standard_normal((k + 1, n))
    sigma = 2.6
    via_forward = W @ O.sweep(Wi @ g, (n,), k, 0, -sigma)
    assert np.allclose(O.sweep_adjoint(g, (n,), k, 0, sigma), via_forward, atol=1e-13, rtol=0)
    # the magnitude form: |W F W^-1| = W |F| W^-1 for the positive diagonal W,
    # so the absolute transpose equals the weight-conjugated absolute forward
    # sweep with the opposite displacement, and bounds the transpose itself
    mag = O.sweep_adjoint(g, (n,), k, 0, sigma, absolute=True)
    via_abs = W @ O.sweep(Wi @ np.abs(g), (n,), k, 0, -sigma, absolute=True)
    assert np.allclose(mag, via_abs, atol=1e-13, rtol=0)
    assert np.all(mag >= np.abs(O.sweep_adjoint(g, (n,), k, 0, sigma)) - 1e-15)


# --------------------------------------------------------------------------
# number of leading coefficients in FP64 (section III-A, Table II axis)
# --------------------------------------------------------------------------

def test_fp64_modes_follow_total_degree():
    keep = O.fp64_modes(2, 2, 2)          # 2D, k = 2: modes with j0 + j1 < 2
    assert [m for m in range(9) if keep[m]] == [0, 1, 3]
    assert O.fp64_modes(1, 3, 4).all() and not O.fp64_modes(3, 1, 0).any()
    assert list(O.fp64_modes(1, 3, 2)) == [1, 1, 0, 0]


def test_all_fp64_modes_equal_the_fp64_tier():
    k, ns = 2, (9, 7)
    rng = np.random.default_rng(17)
    state = rng.standard_normal((9, 63))
    sig = rng.uniform(-3, 3, 7)
    a = O.sweep(state, ns, k, 0, sig, (1,), "fp32", ndouble=2 * k + 1)
    b = O.sweep(state, ns, k, 0, sig, (1,), "fp64")
    assert np.array_equal(a, b)


@pytest.mark.parametrize("ndouble,tier", [(0, "fp32"), (1, "fp32"), (2, "fp32"), (1, "bf16")])
def test_mass_is_conserved_iff_the_cell_mean_is_fp64(ndouble, tier):
    # section III-A: with c_0 in double precision the mass is conserved to
    # double precision; with every coefficient in single precision it is not
    n, k, steps = 64, 3, 3000
    rng = np.random.default_rng(1603)
    m = np.arange(1, n // 4 + 1)
    r = rng.uniform(0, 1, m.size) / m
    ph = rng.uniform(0, 2 * np.pi, m.size)
    f = lambda x: 1.0 + np.sum(r[:, None, None] * np.sin(2 * np.pi * m[:, None, None] * x[None] + ph[:, None, None]), axis=0)
    c = O.to_tier(O.project_1d(f, n, 0.0, 1.0, k), tier, ndouble, k=k, ndim=1)
    M0 = O.mass(c, (n,), (0.0,), (1.0,))
    for _ in range(steps):
        c = O.sweep(c, (n,), k, 0, 0.37, tier=tier, ndouble=ndouble)
    drift = abs(O.mass(c, (n,), (0.0,), (1.0,)) - M0) / abs(M0)
    if ndouble >= 1:
        assert drift <= 1e-14
    else:
        assert drift >= 1e-10
