"""Seeded synthetic workloads of the sLdG projection sweep.

This module only describes problems: grids, domains, time steps, initial
functions, displacement fields and seeded random data.  It holds none of the
method's arithmetic (no projection, no update), so both the HIP path and the
CPU oracle can take their inputs from it.

Physics (section II): the Vlasov equation f_t + v f_x + E(x) f_v = 0 is split
(Cheng-Knorr) into advections in x with speed v and in v with speed E(x).  A
sweep along dimension d displaces every line (fixed transverse cell) by
sigma = a * dt / h_d cells, with a evaluated at the transverse cell centre.
"""
import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Sweep:
    dim: int                 # swept dimension (0 = fastest)
    sigma: np.ndarray        # displacement in cells, one per line, over `dep`
    dep: tuple               # dimensions the displacement depends on

    @property
    def dep_mask(self):
        m = 0
        for e in self.dep:
            m |= 1 << e
        return m


@dataclass
class Problem:
    name: str
    ns: tuple                # cells per dimension, dimension 0 fastest
    los: tuple
    his: tuple
    k: int
    steps: int
    seq: list = field(default_factory=list)     # sweeps of one split step
    f0_terms: list = field(default_factory=list)  # f0 = sum_t prod_e f_{t,e}(x_e)

    @property
    def ndim(self):
        return len(self.ns)

    @property
    def cells(self):
        return int(np.prod(self.ns))

    @property
    def modes(self):
        return (self.k + 1) ** self.ndim

    @property
    def h(self):
        return tuple((self.his[e] - self.los[e]) / self.ns[e] for e in range(self.ndim))

    def centres(self, e):
        return self.los[e] + (np.arange(self.ns[e]) + 0.5) * self.h[e]

    @property
    def coeff_updates_per_step(self):
        return len(self.seq) * self.cells * self.modes


def maxwellian(v):
    return np.exp(-0.5 * v * v) / math.sqrt(2.0 * math.pi)


def _grid_field(prob, dep, fn):
    """fn evaluated at the cell centres of the dims in `dep`, flattened with the
    lowest dimension fastest."""
    axes = [prob.centres(e) for e in sorted(dep)]
    if not axes:
        return np.atleast_1d(np.float64(fn()))
    grids = np.meshgrid(*axes, indexing="ij")        # grids[i] varies along axis i
    val = fn(*grids)
    # flatten with the first listed (lowest) dimension fastest
    return np.ascontiguousarray(np.asarray(val, dtype=np.float64).transpose(
        tuple(range(len(axes) - 1, -1, -1)))).ravel()


def advection_1d(n=64, k=2, sigma=0.37, steps=270):
    """u_t + u_x = 0 on [0, 1), u0 = sin(2 pi x), displacement sigma cells/step."""
    p = Problem("advection-1d", (n,), (0.0,), (1.0,), k, steps)
    p.seq = [Sweep(0, np.array([sigma]), ())]
    p.f0_terms = [(lambda x: np.sin(2 * np.pi * x),)]
    return p


def vlasov_2d(nx=256, nv=256, k=2, dt=0.1, steps=200, eps=0.01):
    """2D (x, v): x in [0, 4 pi) periodic, v in [-6, 6) periodic,
    f0 = (1 + eps cos(x/2)) M(v), E(x) = eps sin(x/2)/0.5; Strang splitting
    X(dt/2) V(dt) X(dt/2)."""
    p = Problem("vlasov-2d", (nx, nv), (0.0, -6.0), (4 * math.pi, 6.0), k, steps)
    hx, hv = p.h
    sx = _grid_field(p, (1,), lambda v: v * (0.5 * dt) / hx)
    sv = _grid_field(p, (0,), lambda x: eps * np.sin(0.5 * x) / 0.5 * dt / hv)
    p.seq = [Sweep(0, sx, (1,)), Sweep(1, sv, (0,)), Sweep(0, sx, (1,))]
    p.f0_terms = [(lambda x: 1.0 + eps * np.cos(0.5 * x), maxwellian)]
    return p


def efield_4d(seed=1603, amp=0.005):
    """Seeded smooth periodic E(x1, x2) = (E1, E2) on [0, 4 pi)^2:
    E_d = sum_{(m,n) in {0,1,2}^2, (m,n) != 0} a_mn sin((m x1 + n x2)/2 + phi_mn)."""
    rng = np.random.default_rng(seed)
    modes = [(m, n) for m in range(3) for n in range(3) if (m, n) != (0, 0)]
    a = rng.uniform(-amp, amp, size=(2, len(modes)))
    phi = rng.uniform(0.0, 2 * math.pi, size=(2, len(modes)))

    def E(d, x1, x2):
        out = np.zeros(np.broadcast(x1, x2).shape)
        for q, (m, n) in enumerate(modes):
            out += a[d, q] * np.sin(0.5 * (m * x1 + n * x2) + phi[d, q])
        return out
    return E


def vlasov_4d(n=48, k=2, dt=0.1, steps=20, ns=None, seed=1603):
    """4D (x1, x2, v1, v2): x in [0, 4 pi)^2, v in [-6, 6)^2, all periodic,
    f0 = (1 + 0.01 cos(x1/2) + 0.01 cos(x2/2)) M(v1) M(v2), seeded smooth E;
    split step X1(dt/2) X2(dt/2) V1(dt) V2(dt) X1(dt/2) X2(dt/2)."""
    ns = (n, n, n, n) if ns is None else tuple(ns)
    p = Problem("vlasov-4d", ns, (0.0, 0.0, -6.0, -6.0),
                (4 * math.pi, 4 * math.pi, 6.0, 6.0), k, steps)
    h = p.h
    E = efield_4d(seed)
    sx1 = _grid_field(p, (2,), lambda v1: v1 * (0.5 * dt) / h[0])
    sx2 = _grid_field(p, (3,), lambda v2: v2 * (0.5 * dt) / h[1])
    sv1 = _grid_field(p, (0, 1), lambda x1, x2: E(0, x1, x2) * dt / h[2])
    sv2 = _grid_field(p, (0, 1), lambda x1, x2: E(1, x1, x2) * dt / h[3])
    X1, X2 = Sweep(0, sx1, (2,)), Sweep(1, sx2, (3,))
    p.seq = [X1, X2, Sweep(2, sv1, (0, 1)), Sweep(3, sv2, (0, 1)), X1, X2]
    one = lambda x: np.ones_like(x)
    p.f0_terms = [
        (one, one, maxwellian, maxwellian),
        (lambda x: 0.01 * np.cos(0.5 * x), one, maxwellian, maxwellian),
        (one, lambda x: 0.01 * np.cos(0.5 * x), maxwellian, maxwellian),
    ]
    return p


def random_coefficients(ndim, k, cells, seed=0, scale0=0.15, decay=0.05):
    """Seeded synthetic coefficients with the magnitude profile of smooth
    Vlasov data: mode (j_0, ..., j_{d-1}) has rms scale0 * decay^(sum j).
    Returns float64 [o^ndim, cells]."""
    rng = np.random.default_rng(seed)
    o = k + 1
    M = o ** ndim
    out = np.empty((M, cells))
    for m in range(M):
        js = sum((m // o ** e) % o for e in range(ndim))
        if m == 0:
            out[m] = scale0 * (1.0 + 0.1 * rng.standard_normal(cells))
        else:
            out[m] = scale0 * decay ** js * rng.standard_normal(cells)
    return out


def random_displacements(n, lo, hi, seed=0):
    """Seeded uniform displacements in [lo, hi) cells."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=n)


def random_coefficients_device(ndim, k, cells, seed=0, scale0=0.15, decay=0.05, device="cuda"):
    """The recipe of random_coefficients drawn on the device with torch's
    seeded generator (for grids too large to draw on the host quickly).
    Returns float64 mass [cells] and float64 higher modes [o^ndim - 1, cells]."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    o = k + 1
    M = o ** ndim
    mass = scale0 * (1.0 + 0.1 * torch.randn(cells, generator=g, device=device, dtype=torch.float64))
    hi = torch.empty((M - 1, cells), device=device, dtype=torch.float64)
    for m in range(1, M):
        js = sum((m // o ** e) % o for e in range(ndim))
        hi[m - 1].normal_(0.0, scale0 * decay ** js, generator=g)
    return mass, hi


def vlasov_2d_differentiation(n=512, steps=50, k=2, seed=5, dt=0.1, eps=0.01):
    """The 2D (x, v) problem of vlasov_2d on n x n cells for differentiation:
    fixed E, `steps` Strang steps, and a seeded target
    f_t = (1 + eps cos(x/2 + phi)) M(v) (phi from `seed`), whose projection plus
    N(0, 1e-4) noise on every coefficient (also from `seed`) is the target
    state of the misfit."""
    p = vlasov_2d(nx=n, nv=n, k=k, dt=dt, steps=steps, eps=eps)
    p.name = "vlasov-2d-adjoint"
    rng = np.random.default_rng(seed)
    phi = float(rng.uniform(0.0, 2 * math.pi))
    p.target_terms = [(lambda x: 1.0 + eps * np.cos(0.5 * x + phi), maxwellian)]
    p.target_noise = rng.standard_normal((p.modes, p.cells)) * 1e-4
    return p


def fd_directions(count, modes, cells, seed=6):
    """Seeded N(0, 1) directions over all coefficients, [count, modes, cells]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((count, modes, cells))


def landau_2d(nx, nv, k, dt, kappa, eps=0.01, amp=0.01, steps=1):
    """2D (x, v) Landau-like problem: x in [0, 2 pi / kappa) periodic,
    v in [-6, 6) periodic, f0 = (1 + eps cos(kappa x)) M(v),
    E(x) = amp sin(kappa x) / kappa; Strang X(dt/2) V(dt) X(dt/2)."""
    p = Problem("landau-2d", (nx, nv), (0.0, -6.0), (2 * math.pi / kappa, 6.0), k, steps)
    hx, hv = p.h
    sx = _grid_field(p, (1,), lambda v: v * (0.5 * dt) / hx)
    sv = _grid_field(p, (0,), lambda x: amp * np.sin(kappa * x) / kappa * dt / hv)
    p.seq = [Sweep(0, sx, (1,)), Sweep(1, sv, (0,)), Sweep(0, sx, (1,))]
    p.f0_terms = [(lambda x: 1.0 + eps * np.cos(kappa * x), maxwellian)]
    p.dt, p.kappa = dt, kappa
    return p


def batched_landau(nprob=512, seed=4, nmin=32, nmax=512):
    """Independent Landau-like problems with seeded Nx, Nv ~ U{nmin..nmax},
    k ~ U{1, 2, 3}, dt ~ U[0.02, 0.2], kappa ~ U[0.3, 0.8]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nprob):
        nx, nv = (int(v) for v in rng.integers(nmin, nmax + 1, size=2))
        k = int(rng.integers(1, 4))
        dt = float(rng.uniform(0.02, 0.2))
        kappa = float(rng.uniform(0.3, 0.8))
        out.append(landau_2d(nx, nv, k, dt, kappa))
    return out
