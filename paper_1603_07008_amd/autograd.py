"""Reverse-mode differentiation through split steps of the sLdG sweep.

The split step (section II: Cheng-Knorr splitting into 1D advections) is a
linear map of the coefficients for given displacement fields, so its
gradient is the product of the transposed sweeps in reverse order; each
transposed sweep runs in the library's HIP kernels (sldg_advect_dim_adjoint).
This module only orders the calls and manages buffers.

Checkpointing: with `checkpoint_every = C`, the forward pass keeps the state
at the start of every C-th step.  The backward pass walks the segments from
the last to the first.  With fixed fields (the default) the transposed sweeps
need no forward state and the checkpoints are not read, so the gradient is
bitwise the same with or without them.

Frozen fields (`frozen_shifts_fn`): the displacements of each step may be
computed from the state at the start of the step (a self-consistent field).
The gradient then treats those displacements as constants: it is the
transposed product of the sweeps the forward pass ran, i.e. the derivative
at frozen fields, and not the gradient of the self-consistent map (which
would add the field solve's transpose and the derivatives of A and B with
respect to the displacement).  With checkpoints the backward pass rebuilds
each segment's fields from its checkpoint by re-running the segment forward;
without them the forward pass keeps every step's fields.
"""
import torch

from . import Plan, hi_dtype


class _SplitSteps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mass, hi, plan, seq, nsteps, checkpoint_every, frozen_shifts_fn):
        cur = [(mass.detach().clone(), hi.detach().clone()), plan.empty_state()]
        idx = 0
        ckpts = []
        seqs = []
        for n in range(nsteps):
            if checkpoint_every and n % checkpoint_every == 0:
                ckpts.append((n, cur[idx][0].clone(), cur[idx][1].clone()))
            step_seq = seq if frozen_shifts_fn is None else frozen_shifts_fn(cur[idx])
            if frozen_shifts_fn is not None and not checkpoint_every:
                seqs.append(step_seq)
            res = plan.split_steps(step_seq, 1, cur[idx], cur[1 - idx])
            idx = idx if res == 0 else 1 - idx
        ctx.plan = plan
        ctx.seq = seq
        ctx.nsteps = nsteps
        ctx.checkpoint_every = checkpoint_every
        ctx.checkpoints = ckpts
        ctx.shifts_fn = frozen_shifts_fn
        ctx.seqs = seqs
        return cur[idx][0], cur[idx][1]

    @staticmethod
    def backward(ctx, g_mass, g_hi):
        plan = ctx.plan
        g = (g_mass.detach().contiguous().clone(),
             g_hi.detach().to(hi_dtype(plan.tier)).contiguous().clone())
        tmp = plan.empty_state()

        def adjoint_step(step_seq):
            nonlocal g, tmp
            for dim, mask, shift in reversed(step_seq):
                plan.advect_dim_adjoint(dim, shift, mask, g[0], g[1], tmp[0], tmp[1])
                g, tmp = tmp, g

        if ctx.shifts_fn is None:
            for _ in range(ctx.nsteps):
                adjoint_step(ctx.seq)
        elif not ctx.checkpoint_every:
            for step_seq in reversed(ctx.seqs):
                adjoint_step(step_seq)
        else:
            bounds = [n for n, _, _ in ctx.checkpoints] + [ctx.nsteps]
            for seg in range(len(ctx.checkpoints) - 1, -1, -1):
                n0, m0, h0 = ctx.checkpoints[seg]
                seg_seqs = []
                st = [(m0.clone(), h0.clone()), plan.empty_state()]
                idx = 0
                for _ in range(n0, bounds[seg + 1]):
                    step_seq = ctx.shifts_fn(st[idx])
                    seg_seqs.append(step_seq)
                    res = plan.split_steps(step_seq, 1, st[idx], st[1 - idx])
                    idx = idx if res == 0 else 1 - idx
                for step_seq in reversed(seg_seqs):
                    adjoint_step(step_seq)
        return g[0], g[1], None, None, None, None, None


def split_steps(plan: Plan, seq, nsteps, mass, hi, checkpoint_every=None, frozen_shifts_fn=None):
    """Differentiable split steps: returns (mass, hi) after `nsteps` steps of
    the sweeps `seq` [(dim, dep_mask, shift tensor), ...]; gradients flow to
    `mass` and `hi` through the transposed sweeps.  frozen_shifts_fn(state)
    -> seq, if given, supplies each step's sweeps from the state at the start
    of the step, and the gradient holds those displacements fixed (the
    derivative at frozen fields; see the module docstring)."""
    return _SplitSteps.apply(mass, hi, plan, seq, nsteps, checkpoint_every, frozen_shifts_fn)


def weighted_l2_misfit(mass, hi, t_mass, t_hi, ndim, k, cell_volume):
    """L = 1/2 ||f_h - f_t||^2_{L2} of two piecewise-Legendre states (torch
    ops; differentiable): (prod h)/2 * sum_m w_m sum_cells (c_m - t_m)^2 with
    w_m = prod_e 1/(2 j_e + 1)."""
    o = k + 1
    M = o ** ndim
    w = torch.ones(M, dtype=torch.float64, device=mass.device)
    for m in range(M):
        for e in range(ndim):
            w[m] /= 2 * ((m // o ** e) % o) + 1
    dm = mass - t_mass
    dh = hi.to(torch.float64) - t_hi.to(torch.float64)
    return 0.5 * cell_volume * (w[0] * torch.sum(dm * dm) +
                                torch.sum(w[1:, None] * dh.reshape(M - 1, -1) ** 2))
