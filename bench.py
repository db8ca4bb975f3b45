#!/usr/bin/env python3
"""Benchmark of the MI355X sLdG projection sweep.

Workload: the 4D split-advection problem (x1, x2, v1, v2), 48^4 cells, degree
k = 2 (81 Legendre coefficients per cell, ~430M coefficients), periodic,
seeded synthetic coefficients with the magnitude profile of smooth Vlasov
data and the displacement fields of the 4D Vlasov configuration (x-shifts
v*dt/2, v-shifts E(x1,x2)*dt with a seeded smooth E).  One step = one split
step X1(dt/2) X2(dt/2) V1(dt) V2(dt) X1(dt/2) X2(dt/2) (six sweeps, the
per-line shift tables of each sweep, ping-pong buffers) plus the compensated
mass reduction, i.e. every stage of the hot path.  Inputs are resident in HBM
before timing starts.

Metric: coefficient updates per second (each coefficient of the grid is
rewritten once per sweep), with the achieved HBM bandwidth of the dominant
sweep kernel against the 8 TB/s peak, the FP64 and BF16 tiers timed on the
same data for the mixed-vs-FP64 speedup, and the CPU oracle timed on a
sampled subset of the same step as the baseline.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TIER_BYTES = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2}
ARITH = {"fp64": "f64", "fp32": "f64", "bf16": "f32", "fp16": "f32"}
KERNEL_SOURCES = ["paper_1603_07008_amd/csrc/sldg_kernels.hip", "paper_1603_07008_amd/csrc/ab_poly.h",
                  "paper_1603_07008_amd/csrc/sldg_internal.h", "paper_1603_07008_amd/csrc/sldg_sweep.h",
                  "paper_1603_07008_amd/csrc/sldg_sweep_inst.hip", "paper_1603_07008_amd/csrc/sldg_fused.h",
                  "paper_1603_07008_amd/csrc/sldg_staged.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_vlasov4d_48_k2.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def state_bytes(cells, modes, tier):
    return cells * (8 + TIER_BYTES[tier] * (modes - 1))


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken on the current kernel sources (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    ent = rec.get("kernels", {}).get(kernel)
    return None if ent is None else ent.get("bytes_per_launch")


def measured_copy_bandwidth(sl, torch, nbytes, reps=10):
    """Read+write bandwidth of the library's plain 16-byte-per-thread device
    copy of `nbytes` (the copy-benchmark reference, cf. the paper's Table I)."""
    n = nbytes // 16
    src = torch.ones(n, 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        sl.device_copy(src, dst)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        sl.device_copy(src, dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * n * 16 / (ms * 1e-3) / 1e9


def measured_plane_copy(sl, torch, cells, nplanes, tiers=(1, 3, 9, 27), reps=10):
    """Bandwidth of copying nplanes FP32 planes of `cells` values with 16 B
    per thread, each thread walking T planes in turn: the access pattern of a
    sweep thread's run of spectator tuples, without arithmetic."""
    pb = cells * 4 // 16 * 16
    src = torch.ones(nplanes * pb // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for T in tiers:
        for _ in range(3):
            sl.device_plane_copy(src, dst, pb, nplanes, T)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            sl.device_plane_copy(src, dst, pb, nplanes, T)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[str(T)] = round(2 * pb * nplanes / (ms * 1e-3) / 1e9, 1)
    del src, dst
    return out


def sweep_kernel_name(ns, k, tier, d, shape, form=None):
    """The template instance the library launches for the sweep along d (as
    the profiler names it; `form` as sldg_plan_sweep_form reports it): the
    window or lane form along dimension 0; the staged strided kernel with its
    rows per thread and column waves; the strided kernel with its rows per
    thread and which of its one-value-per-lane stores carry the non-temporal
    hint (where a wave's stores cover whole 128-byte lines: the column stride
    P is a multiple of 64, or P times the value size a multiple of 128
    bytes): 0 none, 1 the 4- and 8-byte values, 2 the 2-byte values too."""
    tid = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3}[tier]
    if form == "staged":
        return (f"sldg::sweep_staged_kernel<{k}, {tid}, {shape['rows']}, "
                f"{shape['colwaves'] & 7}, {1 if tier == 'fp32' else 2}>")
    if d == 0:
        if ns[0] % 4 == 0:
            return f"sldg::sweep_contig_window_kernel<{k}, {tid}, 1>"
        if shape["rows"] in (2, 4, 8):
            return f"sldg::sweep_contig_group_kernel<{k}, {tid}, 1>"
        return f"sldg::sweep_lane_kernel<{k}, {tid}, 1, 2>"
    if shape["rows"] == 0:
        return f"sldg::sweep_lane_kernel<{k}, {tid}, 1, 2>"
    P = 1
    for e in range(d):
        P *= ns[e]
    ok = lambda size: P % 64 == 0 or (P * size) % 128 == 0
    if tier == "fp64":
        nt = 1 if ok(8) else 0
    elif tier == "fp32":
        nt = 1 if ok(4) else 0
    else:
        nt = 2 if ok(2) else (1 if ok(8) else 0)
    rows = shape["rows"]
    while rows > 1 and rows > ns[d]:
        rows //= 2
    return f"sldg::sweep_strided_kernel<{k}, {tid}, {rows}, 1, {nt}>"


def run_tier(sl, torch, prob, tier, init, steps, warmup, tune_cache=None, single_reps=20, settle=10):
    """Time `steps` split steps (after `warmup`) of `prob` in `tier`: the
    split step as the library runs it (the (x1, x2) sweep pairs fused into one
    pass each), then the same steps with every sweep its own pass (the
    per-sweep figures)."""
    p = sl.Plan(prob.ns, prob.k, tier)
    mass0, hi0 = init
    s0 = (mass0.clone(), hi0.to(sl.hi_dtype(tier), copy=True).contiguous())
    s1 = p.empty_state()
    seq = [(sw.dim, sw.dep_mask, torch.from_numpy(sw.sigma).cuda()) for sw in prob.seq]
    mout = torch.zeros(2, dtype=torch.float64, device="cuda")
    bufs = [s0, s1]
    cur = 0

    def step():
        nonlocal cur
        res = p.split_steps(seq, 1, bufs[cur], bufs[1 - cur])
        cur = cur if res == 0 else 1 - cur
        p.mass_device(bufs[cur][0], mout)

    # launch shapes: the plan's autotuner, once, outside the timed region
    # (or shapes tuned earlier, from a JSON cache)
    if tune_cache:
        shapes, _ = p.tune_cached(tune_cache, seq, s0, s1, reps=3)
    else:
        shapes, _ = p.tune(seq, s0, s1, reps=3)
    tid = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3}[tier]
    forms = {d: p.sweep_form(d, dep, s0, s1) for d, dep, _ in seq}
    out = {"plan": p, "shapes": shapes, "forms": forms}
    m_start = p.mass(bufs[cur][0])
    for fuse in (True, False):
        p.set_fusion(fuse)
        # untimed settling steps before the warm-up: after the tuner's
        # memory-bound launches the fused pass (busier ALUs) takes about 15
        # launches to reach its steady duration (kernel trace: 0.85-0.91 ms
        # falling to 0.65 ms)
        for _ in range(settle + warmup):
            step()
        torch.cuda.synchronize()
        p.timing_enable(True)
        ev0, ev1 = _events(torch)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(steps):
            step()
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        per_dim = {d: p.timing_read(d) for d in range(prob.ndim)}
        fused = p.timing_read(-3)
        p.timing_enable(False)
        kern = {}                   # kernel (template instance) -> (launches, total ms)
        for d, (n, tot) in per_dim.items():
            if n:
                name = sweep_kernel_name(prob.ns, prob.k, tier, d, shapes[d], forms[d])
                n0, t0 = kern.get(name, (0, 0.0))
                kern[name] = (n0 + n, t0 + tot)
        if fused[0]:
            kern[f"sldg::sweep_xy_kernel<{prob.k}, {tid}>"] = fused
        key = "fused" if fuse else "unfused"
        out[key] = {"ms_per_step": ms, "kernels": kern, "per_dim": per_dim, "fused": fused}
    p.set_fusion(True)
    out["steps_run"] = 2 * (settle + warmup + steps)
    m_end = p.mass(bufs[cur][0])
    out["mass_drift"] = abs((m_end[0] + m_end[1]) - (m_start[0] + m_start[1])) / \
        abs(m_start[0] + m_start[1])
    out["ms_per_step"] = out["fused"]["ms_per_step"]
    out["final"] = bufs[cur]
    # each sweep direction alone (its table launch included): event pairs
    # around single calls, after 3 warm-ups, outside the timed steps
    single = {}
    final, other = bufs[cur], bufs[1 - cur]
    for d, dep, sig in seq:
        if d in single:
            continue
        for _ in range(3):
            p.advect_dim(d, sig, dep, *final, *other)
        ts = []
        for _ in range(single_reps):
            e0, e1 = _events(torch)
            e0.record()
            p.advect_dim(d, sig, dep, *final, *other)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ts.sort()
        single[d] = {"median_ms": round(ts[len(ts) // 2], 4), "min_ms": round(ts[0], 4),
                     "reps": single_reps}
    out["single"] = single
    return out


def oracle_errors(sl, torch, prob, tier, mass0, hi0, ncheck, seed):
    """One sweep per direction, and the fused (x1, x2) pass, from the
    benchmark's initial state rounded to `tier`, against the FP64 oracle from
    the same state: relative L2 error in the mode-weighted norm over
    `ncheck` sampled output cells, and the largest relative error of the FP64
    mass mode."""
    import numpy as np
    from oracle import sldg_oracle as O
    modes, cells = prob.modes, prob.cells
    scaled = tier == "fp16_scaled"
    p = sl.Plan(prob.ns, prob.k, "fp16" if scaled else tier)
    if scaled:
        # FP16 planes with per-plane power-of-two scales, imported from FP64
        h16 = torch.empty((p.n_hi, p.cells), dtype=torch.float16, device="cuda")
        sc = p.empty_scale()
        p.scaled_import(hi0, h16, sc)
        a = (mass0, h16, sc)
        b = (*p.empty_state(), p.empty_scale())
        hi_vals = p.scaled_export(h16, sc)
    else:
        hi_t = hi0.to(sl.hi_dtype(tier)).contiguous()
        a = (mass0, hi_t)
        b = p.empty_state()
        hi_vals = hi_t.to(torch.float64)
    host = np.empty((modes, cells))
    host[0] = mass0.cpu().numpy()
    host[1:] = hi_vals.cpu().numpy().reshape(modes - 1, cells)
    del hi_vals
    rng = np.random.default_rng(seed)
    probe = np.sort(rng.choice(cells, min(cells, ncheck), replace=False))
    idx = torch.from_numpy(probe).cuda()
    w = O.mode_weights(prob.ndim, prob.k)[:, None]

    def gathered(state):
        got = np.empty((modes, probe.size))
        got[0] = state[0][idx].cpu().numpy()
        h = p.scaled_export(state[1], state[2]) if scaled else state[1].reshape(modes - 1, cells)
        got[1:] = h[:, idx].to(torch.float64).cpu().numpy()
        return got

    def sweep(dim, sig, mask):
        if scaled:
            p.advect_dim_scaled(dim, sig, mask, *a, *b)
        else:
            p.advect_dim(dim, sig, mask, *a, *b)

    def compare(got, want):
        rel = math.sqrt(float(np.sum(w * (got - want) ** 2)) / float(np.sum(w * want ** 2)))
        return {"rel_l2_vs_oracle_fp64": rel,
                "mass_mode_max_rel_err": float(np.max(np.abs(got[0] - want[0]) / np.abs(want[0])))}

    names = {0: "X1", 1: "X2", 2: "V1", 3: "V2"}
    res = {}
    done = set()
    for sw in prob.seq:
        if sw.dim in done:
            continue
        done.add(sw.dim)
        sweep(sw.dim, torch.from_numpy(sw.sigma).cuda(), sw.dep_mask)
        want = O.sweep(host, prob.ns, prob.k, sw.dim, sw.sigma, sw.dep, "fp64", sel=probe)
        res[names.get(sw.dim, str(sw.dim))] = compare(gathered(b), want)
    # the fused pair: the oracle's x1 sweep on the cells the x2 sweep of the
    # sampled cells reads, then its x2 sweep
    sx1, sx2 = prob.seq[0], prob.seq[1]
    if scaled:                      # no fused pass for scaled storage: two sweeps
        mid_state = (*p.empty_state(), p.empty_scale())
        p.advect_dim_scaled(0, torch.from_numpy(sx1.sigma).cuda(), sx1.dep_mask, *a, *mid_state)
        p.advect_dim_scaled(1, torch.from_numpy(sx2.sigma).cuda(), sx2.dep_mask, *mid_state, *b)
        del mid_state
    else:
        p.advect_dims01(torch.from_numpy(sx1.sigma).cuda(), sx1.dep_mask,
                        torch.from_numpy(sx2.sigma).cuda(), sx2.dep_mask, *a, *b)
    got = gathered(b)
    n0, n1 = prob.ns[0], prob.ns[1]
    i1 = (probe // n0) % n1
    base = probe - i1 * n0
    s_tab, _ = O.line_tables(sx2.sigma, prob.k)
    # the line of each sampled cell in the x2 sweep's table (over the
    # dimensions its displacement depends on, lowest fastest)
    line = np.zeros(probe.size, dtype=np.int64)
    stride = 1
    for e in sx2.dep:
        line += ((probe // int(np.prod(prob.ns[:e]))) % prob.ns[e]) * stride
        stride *= prob.ns[e]
    s = s_tab[line].astype(np.int64)
    src = np.concatenate([base + ((i1 - s) % n1) * n0, base + ((i1 - s - 1) % n1) * n0])
    need = np.unique(src)
    mid_sel = O.sweep(host, prob.ns, prob.k, sx1.dim, sx1.sigma, sx1.dep, "fp64", sel=need)
    mid = np.zeros_like(host)
    mid[:, need] = mid_sel
    del host
    want = O.sweep(mid, prob.ns, prob.k, sx2.dim, sx2.sigma, sx2.dep, "fp64", sel=probe)
    res["X1X2 two sweeps" if scaled else "X1X2 fused"] = compare(got, want)
    p.close()
    del b, mid
    res["cells"] = int(probe.size)
    return res


def cpu_baseline(prob, tier, seconds, seed, state=None):
    """The CPU oracle timed on a sampled subset of one split step: the full
    4D state in host memory (the benchmark's initial state when given),
    every sweep of the step computed for the same random sample of output
    cells (all 81 coefficients of each), once with the oracle's OpenMP
    threads and once on one thread, so the two rates are taken at the same
    sample density.  The sample is sized for about `seconds` of one-thread
    work."""
    import numpy as np
    from oracle import sldg_oracle as O
    from paper_1603_07008_amd import inputs
    t0 = time.time()
    if state is None:
        state = O.to_tier(inputs.random_coefficients(prob.ndim, prob.k, prob.cells, seed=seed), tier)
    log(f"cpu_baseline: host state ready in {time.time() - t0:.1f}s")
    rng = np.random.default_rng(seed + 1)
    for sw in prob.seq:                   # the oracle's A/B cache, outside the timing
        O.line_tables(sw.sigma, prob.k)

    def timed(sel):
        t = time.perf_counter()
        for sw in prob.seq:
            O.sweep(state, prob.ns, prob.k, sw.dim, sw.sigma, sw.dep, tier, sel=sel)
        return time.perf_counter() - t

    nt = O.num_threads()
    O.set_threads(1)
    try:
        cal = np.sort(rng.choice(prob.cells, min(prob.cells, 8192), replace=False))
        per = timed(cal) / cal.size           # one-thread seconds per sampled cell (upper bound)
        nsel = int(min(prob.cells, max(8192, seconds / per)))
        sel = np.sort(rng.choice(prob.cells, nsel, replace=False))
        dt1 = timed(sel)
    finally:
        O.set_threads(nt)
    dt = timed(sel)
    updates = nsel * prob.modes * len(prob.seq)
    cores = len(os.sched_getaffinity(0))
    return {"value": updates / dt, "unit": "coeff-updates/s", "cores": nt,
            "host_cpus_available": cores,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"),
            "kind": "oracle", "value_1_thread": updates / dt1,
            "sample": f"one split step (6 sweeps) of the {prob.ns} k={prob.k} {tier}-mode "
                      f"workload on the full host state, evaluated for the same {nsel} randomly "
                      f"sampled output cells x {prob.modes} coefficients ({updates} coefficient "
                      f"updates) on {nt} OpenMP threads ({dt:.2f} s) and on one thread "
                      f"({dt1:.1f} s)"}


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def batched_extra(sl, torch, steps, seed):
    """The batched workload: 512 independent (x, v) problems of seeded extents
    32..512 and degrees 1..3 in FP32-mode, one persistent launch per sweep,
    launch shapes from the batch tuner; eager launches and HIP-graph replays
    of the split step."""
    from paper_1603_07008_amd import inputs
    from paper_1603_07008_amd.batch import Batch
    probs = inputs.batched_landau(nprob=512, seed=4)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = Batch([p.ns for p in probs], [p.k for p in probs], "fp32", stream=stream.cuda_stream)
        s0, s1 = [], []
        for i, p in enumerate(probs):
            m, h = inputs.random_coefficients_device(2, p.k, p.cells, seed=seed + i)
            s0.append((m, h.to(torch.float32)))
            s1.append((torch.empty_like(m), torch.empty_like(s0[-1][1])))
        b.bind(s0, s1)
        shifts = [[(sw.dep_mask, torch.from_numpy(sw.sigma).cuda()) for sw in p.seq] for p in probs]
        b.set_sequence([(probs[0].seq[q].dim, [shifts[i][q] for i in range(len(probs))])
                        for q in range(3)])
        init = [(m.clone(), h.clone()) for m, h in s0]
        tuned = b.tune(reps=2)
        for i in range(len(probs)):                 # the tuner overwrote buffer 1 only
            s0[i][0].copy_(init[i][0])
            s0[i][1].copy_(init[i][1])
        stream.synchronize()
        out = {}
        for mode, graph in (("eager", False), ("graph", True)):
            b.run(2, use_graph=graph)               # warm-up (and graph capture)
            stream.synchronize()
            e0, e1 = _events(torch)
            e0.record(stream)
            b.run(steps, use_graph=graph)
            e1.record(stream)
            stream.synchronize()
            out[mode] = e0.elapsed_time(e1) / steps
    updates = sum(p.cells * p.modes for p in probs) * 3
    sbytes = sum(state_bytes(p.cells, p.modes, "fp32") for p in probs)
    best = min(out.values())
    res = {"workload": "512 Landau-like (x, v) problems, N_x, N_v ~ U{32..512}, k ~ U{1,2,3}, "
                       "fp32-mode, Strang step = 3 sweeps",
           "cells": sum(p.cells for p in probs), "coefficients": sum(p.cells * p.modes for p in probs),
           "ms_per_step_eager": round(out["eager"], 4), "ms_per_step_graph": round(out["graph"], 4),
           "coeff_updates_per_s": updates / (best * 1e-3),
           "algorithmic_GBps": round(3 * 2 * sbytes / (best * 1e-3) / 1e9, 1),
           "frac_hbm_peak": round(3 * 2 * sbytes / (best * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "tuned_shapes": tuned}
    b.close()
    return res


def adjoint_extra(sl, torch, seed):
    """The differentiation workload: 512^2 cells, k = 2, FP64, 50 Strang steps
    forward and the adjoint sweeps backward (checkpoints every 10 steps)."""
    from paper_1603_07008_amd import inputs
    from paper_1603_07008_amd import autograd as AG
    prob = inputs.vlasov_2d_differentiation()
    p = sl.Plan(prob.ns, prob.k, "fp64")
    seq = [(sw.dim, sw.dep_mask, torch.from_numpy(sw.sigma).cuda()) for sw in prob.seq]
    m, h = inputs.random_coefficients_device(2, prob.k, prob.cells, seed=seed)
    tm, th = inputs.random_coefficients_device(2, prob.k, prob.cells, seed=seed + 1)
    vol = 1.0

    def once():
        mm = m.clone().requires_grad_(True)
        hh = h.clone().requires_grad_(True)
        fm, fh = AG.split_steps(p, seq, prob.steps, mm, hh, checkpoint_every=10)
        loss = AG.weighted_l2_misfit(fm, fh, tm, th, 2, prob.k, vol)
        loss.backward()
        return mm.grad, hh.grad

    once()
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    reps = 3
    for _ in range(reps):
        once()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nsw = prob.steps * len(prob.seq)
    return {"workload": "vlasov-2d 512^2, k=2, fp64, 50 Strang steps forward + adjoint backward, "
                        "checkpoints every 10 steps",
            "ms_forward_backward": round(ms, 3),
            "coeff_updates_per_s": 2 * nsw * prob.cells * prob.modes / (ms * 1e-3)}


def scaled_fp16_extra(sl, torch, prob, init, steps, warmup, ref_final, shapes=None, wm=None,
                      total_steps=None, tune_cache=None):
    """The headline 4D step with FP16 storage and per-plane scaling, in
    launch shapes tuned on the FP16 plan itself (its sweeps without the
    scale bookkeeping, outside the timed region), or in `shapes` when given.
    The run continues untimed to `total_steps`, the step count of the other
    tiers' runs, for the comparison with the FP64 run; mode weights `wm`
    give the L2 norm of the piecewise polynomials."""
    p = sl.Plan(prob.ns, prob.k, "fp16")
    mass0, hi0 = init
    m0 = mass0.clone()
    h0 = torch.empty((p.n_hi, p.cells), dtype=torch.float16, device="cuda")
    sc0 = p.empty_scale()
    p.scaled_import(hi0, h0, sc0)
    st = [(m0, h0, sc0), (*p.empty_state(), p.empty_scale())]
    seq = [(sw.dim, sw.dep_mask, torch.from_numpy(sw.sigma).cuda()) for sw in prob.seq]
    if shapes:
        for d, sh in enumerate(shapes):
            p.set_shape(d, sh["rows"], sh["tuples"], sh["colwaves"])
    elif tune_cache:
        p.tune_cached(tune_cache, seq, st[0][:2], st[1][:2], reps=2)
    else:
        p.tune(seq, st[0][:2], st[1][:2], reps=2)
    cur = 0
    m_start = p.mass(m0)
    for _ in range(warmup):
        cur = cur if p.split_steps_scaled(seq, 1, st[cur], st[1 - cur]) == 0 else 1 - cur
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    for _ in range(steps):
        cur = cur if p.split_steps_scaled(seq, 1, st[cur], st[1 - cur]) == 0 else 1 - cur
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    for _ in range(max(0, (total_steps or 0) - warmup - steps)):
        cur = cur if p.split_steps_scaled(seq, 1, st[cur], st[1 - cur]) == 0 else 1 - cur
    m_end = p.mass(st[cur][0])
    out = {"ms_per_step": round(ms, 4),
           "mass_drift_rel": abs((m_end[0] + m_end[1]) - (m_start[0] + m_start[1]))
           / abs(m_start[0] + m_start[1])}
    if ref_final is not None:
        fm = st[cur][0]
        fh = p.scaled_export(st[cur][1], st[cur][2])
        rm, rh = ref_final
        n_hi = fh.shape[0]
        num = wm[0] * torch.sum((fm - rm) ** 2) + \
            torch.sum(wm[1:, None] * (fh - rh.reshape(n_hi, -1)) ** 2)
        den = wm[0] * torch.sum(rm ** 2) + torch.sum(wm[1:, None] * rh.reshape(n_hi, -1) ** 2)
        out["rel_l2_vs_fp64_gpu_run"] = float(torch.sqrt(num / den))
    p.close()
    return out


def next4_extra(sl, torch, prob, init, reps=10):
    """The steps around the path: the 4D x1-sweep with Gauss-node collocation
    in v1 (FP32-mode), and a self-consistent (x, v) Vlasov-Poisson step."""
    out = {}
    p = sl.Plan(prob.ns, prob.k, "fp32")
    mass0, hi0 = init
    s0 = (mass0.clone(), hi0.to(torch.float32).contiguous())
    s1 = p.empty_state()
    sw = prob.seq[0]                                   # x1 sweep, displacement from v1
    o = prob.k + 1
    xi = [float(v) for v in __import__("numpy").polynomial.legendre.leggauss(o)[0]]
    n1 = prob.ns[sw.dep[0]]
    # displacement at the v1 Gauss nodes: linear in v1 across each cell
    sig = torch.from_numpy(sw.sigma).cuda()
    dsig = torch.empty_like(sig)
    dsig[1:-1] = 0.5 * (sig[2:] - sig[:-2])
    dsig[0], dsig[-1] = sig[1] - sig[0], sig[-1] - sig[-2]
    node = (sig[:, None] + 0.5 * dsig[:, None] * torch.tensor(xi, dtype=torch.float64,
                                                             device="cuda")[None, :]).contiguous()
    for _ in range(3):
        p.advect_dim_collocated(sw.dim, sw.dep[0], node, *s0, *s1)
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    for _ in range(reps):
        p.advect_dim_collocated(sw.dim, sw.dep[0], node, *s0, *s1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * state_bytes(prob.cells, prob.modes, "fp32")
    out["collocated_x1_sweep"] = {"ms": round(ms, 4),
                                  "algorithmic_GBps": round(nbytes / (ms * 1e-3) / 1e9, 1),
                                  "frac_hbm_peak": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    p.close()
    from paper_1603_07008_amd import inputs
    pr = inputs.landau_2d(512, 512, 2, 0.1, 0.5)
    q = sl.Plan(pr.ns, pr.k, "fp32")
    m, h = inputs.random_coefficients_device(2, pr.k, pr.cells, seed=7)
    a = (m, h.to(torch.float32).contiguous())
    b = q.empty_state()
    hx, hv = pr.h
    sx = torch.from_numpy(pr.seq[0].sigma).cuda()
    q.vlasov_poisson_steps(2, sx, hx, hv, pr.dt, a, b)
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    q.vlasov_poisson_steps(20, sx, hx, hv, pr.dt, a, b)
    e1.record()
    torch.cuda.synchronize()
    out["vlasov_poisson_step_512x512_k2"] = {"ms_per_step": round(e0.elapsed_time(e1) / 20, 4)}
    q.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tier", default="fp32", choices=list(TIER_BYTES))
    ap.add_argument("--n", type=int, default=48, help="cells per dimension of the 4D grid")
    ap.add_argument("--compare", default="fp64,bf16",
                    help="other tiers timed on the same data (for the speedup)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=1603)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched, adjoint and scaled-FP16 measurements")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON cache of tuned launch shapes (read if it has the plan, else written)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU decomposition is described, not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1603_07008_amd as sl
    from paper_1603_07008_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py: no HIP device", file=sys.stderr)
        sys.exit(1)
    sl.lib()
    prob = inputs.vlasov_4d(n=args.n)
    cells, modes = prob.cells, prob.modes
    log(f"bench: {prob.name} {prob.ns} k={prob.k}: {cells} cells x {modes} coefficients")
    mass0, hi0 = inputs.random_coefficients_device(prob.ndim, prob.k, cells, seed=args.seed)
    torch.cuda.synchronize()

    copy_gbs = measured_copy_bandwidth(sl, torch, state_bytes(cells, modes, args.tier))
    log(f"bench: device copy bandwidth {copy_gbs:.0f} GB/s")
    plane_gbs = measured_plane_copy(sl, torch, cells, modes)
    log(f"bench: plane copy bandwidth by planes per thread {plane_gbs}")
    tiers = [args.tier] + [t for t in args.compare.split(",") if t and t != args.tier]
    results = {}
    for t in tiers:
        log(f"bench: timing tier {t}")
        results[t] = run_tier(sl, torch, prob, t, (mass0, hi0), args.steps, args.warmup,
                              args.tune_cache)
        log(f"bench: {t}: {results[t]['ms_per_step']:.3f} ms/step")

    main_r = results[args.tier]
    ms = main_r["ms_per_step"]
    updates_per_step = len(prob.seq) * cells * modes
    value = updates_per_step / (ms * 1e-3)

    # roofline of the dominant kernel of the step as the library runs it
    # (largest total time); every launch, fused or not, reads and writes the
    # state once
    sbytes = state_bytes(cells, modes, args.tier)
    launch_bytes = 2 * sbytes
    kname, (nl, tot) = max(main_r["fused"]["kernels"].items(), key=lambda kv: kv[1][1])
    avg_ms = tot / max(nl, 1)
    achieved = launch_bytes / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(kname)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": kname, "launches": nl,
                "sweeps_per_launch": 2 if "sweep_xy_kernel" in kname else 1,
                "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": launch_bytes,
                "copy_GBps": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                "plane_copy_GBps": plane_gbs}

    def rate(tot_ms, n):
        a = tot_ms / n
        gbs = launch_bytes / (a * 1e-3) / 1e9
        return {"avg_ms": round(a, 4), "GB/s": round(gbs, 1),
                "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}

    names = {0: "X1", 1: "X2", 2: "V1", 3: "V2"}
    per_sweep = {}                     # every sweep its own pass
    for d, (n, tot_d) in main_r["unfused"]["per_dim"].items():
        if n:
            per_sweep[names.get(d, str(d))] = dict(rate(tot_d, n),
                                                   launch_shape=main_r["shapes"][d],
                                                   form=main_r["forms"][d],
                                                   single_call=main_r["single"].get(d))
    per_pass = {}                      # the step as timed: (x1, x2) pairs fused
    nf, tf = main_r["fused"]["fused"]
    if nf:
        per_pass["X1X2 fused"] = dict(rate(tf, nf), sweeps=2)
    for d, (n, tot_d) in main_r["fused"]["per_dim"].items():
        if n:
            per_pass[names.get(d, str(d))] = dict(rate(tot_d, n), sweeps=1)

    # mixed vs FP64: speedup, and the error of the mixed run against the FP64
    # run after the timed steps (mode-weighted L2 norm, i.e. the L2 norm of the
    # piecewise polynomials)
    o = prob.k + 1
    wm = torch.ones(modes, dtype=torch.float64, device="cuda")
    for m in range(modes):
        for e in range(prob.ndim):
            wm[m] /= 2 * ((m // o ** e) % o) + 1
    tiers_out = {}
    ref = results.get("fp64")
    for t, r in results.items():
        ent = {"ms_per_step": round(r["ms_per_step"], 4),
               "ms_per_step_unfused": round(r["unfused"]["ms_per_step"], 4),
               "coeff_updates_per_s": updates_per_step / (r["ms_per_step"] * 1e-3),
               "bytes_per_update": round(2 * state_bytes(cells, modes, t) / (cells * modes), 3),
               "mass_drift_rel": r["mass_drift"]}
        if ref is not None:
            ent["speedup_vs_fp64"] = round(ref["ms_per_step"] / r["ms_per_step"], 3)
            ent["speedup_vs_fp64_unfused"] = round(ref["unfused"]["ms_per_step"] /
                                                   r["unfused"]["ms_per_step"], 3)
            if t != "fp64":
                fm, fh = r["final"]
                rm, rh = ref["final"]
                num = wm[0] * torch.sum((fm - rm) ** 2) + \
                    torch.sum(wm[1:, None] * (fh.double() - rh).reshape(modes - 1, -1) ** 2)
                den = wm[0] * torch.sum(rm ** 2) + \
                    torch.sum(wm[1:, None] * rh.reshape(modes - 1, -1) ** 2)
                ent["rel_l2_vs_fp64_gpu_run"] = float(torch.sqrt(num / den))
        tiers_out[t] = ent

    out = {
        "metric": "Coefficient updates/s and % HBM peak per sweep; mixed vs FP64 at stated error",
        "value": value,
        "unit": "coeff-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ARITH[args.tier],
        "data": "synthetic (seeded random coefficients, Vlasov magnitude profile; seeded shift fields)",
        "config": {"workload": f"vlasov-4d split step, {args.n}^4 cells, k=2, 81 coeffs/cell, "
                               f"6 sweeps + mass per step",
                   "storage": f"mass f64 + modes {args.tier}", "parallelism": "single GPU",
                   "step": "X1 X2 V1 V2 X1 X2, each (X1, X2) pair as one fused pass"},
        "roofline": roofline,
        "per_pass": per_pass,
        "per_sweep": per_sweep,
        "tiers": tiers_out,
    }
    if not args.no_extras:
        extras = {}
        log("bench: scaled fp16 tier")
        ref = results.get("fp64")
        extras["fp16_scaled"] = scaled_fp16_extra(
            sl, torch, prob, (mass0, hi0), args.steps, args.warmup, ref["final"] if ref else None,
            wm=wm, total_steps=results[args.tier]["steps_run"], tune_cache=args.tune_cache)
        if ref:
            extras["fp16_scaled"]["speedup_vs_fp64"] = round(
                ref["ms_per_step"] / extras["fp16_scaled"]["ms_per_step"], 3)
        out["extras"] = extras
    for r in results.values():
        r["plan"].close()
    results.clear()
    if not args.no_extras:
        log("bench: batched workload")
        extras["batched"] = batched_extra(sl, torch, 20, args.seed)
        log("bench: differentiation workload")
        extras["adjoint"] = adjoint_extra(sl, torch, args.seed)
        log("bench: collocated sweep and self-consistent field")
        extras["next4"] = next4_extra(sl, torch, prob, (mass0, hi0))
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle baseline")
        import numpy as np
        # the benchmark's initial state, rounded to the tier, on the host
        hi_t = hi0.to(sl.hi_dtype(args.tier))
        host = np.empty((modes, cells))
        host[0] = mass0.cpu().numpy()
        host[1:] = hi_t.to(torch.float64).cpu().numpy().reshape(modes - 1, cells)
        del hi_t
        out["cpu_baseline"] = cpu_baseline(prob, args.tier, args.cpu_seconds, args.seed, state=host)
        del host
        # every tier's sweeps against the FP64 oracle from the same initial state
        log("bench: tier errors against the FP64 oracle")
        for t in tiers_out:
            tiers_out[t]["vs_oracle_fp64"] = oracle_errors(sl, torch, prob, t, mass0, hi0, 65536,
                                                          args.seed + 2)
        if not args.no_extras:
            out["extras"]["fp16_scaled"]["vs_oracle_fp64"] = oracle_errors(
                sl, torch, prob, "fp16_scaled", mass0, hi0, 65536, args.seed + 2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
