#!/usr/bin/env python3
"""Throughput of the batched SVGD-FWI hot path on one MI355X.

One step = the whole hot path over one batch: the log-posterior gradient of
every particle (2-D acoustic FD forward with checkpoints, recompute and adjoint
sweeps, imaging, shot sum; vip_grad_logpost) followed by one stochastic SVGD
update of the ensemble (median-bandwidth RBF kernel with the Gram on BF16
matrix cores, kernel-weighted gradients and repulsion, Cholesky-correlated
noise, prior clip; vip_ssvgd_step).

Workload: 200 x 120 cells at 20 m (+ 20-cell sponge), nt = 2000 at 2 ms,
10 shots at 20 m depth, 200 receivers at 360 m, 8 Hz Ricker, 128 particles,
checkpoints every 50 steps; synthetic faulted velocity model, data from the
library's own forward simulation plus 2 % noise, particles from the uniform
prior.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  `value` is particle-gradients per second (one
particle-gradient = one particle's forward + adjoint over all its shots, the
paper's unit of cost); the line also carries the plain per-pair GPU path, the
SVGD step rate at n = 2048, d = 24000, the roofline of the time-stepping
kernel and the FP64 oracle timed on the host as a CPU baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle gradients/s (fwd+adjoint) + SVGD steps/s vs plain path, at stated err"
HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed (dual) FP32 instructions, which the build
# disables: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.
ALU_PEAK_TFLOPS = 78.6
ALU_PUBLISHED_TFLOPS = 157.3
# Streaming-equivalent HBM bytes per padded grid point per pair per time step
# (a "point-step"): what a sweep that keeps nothing on chip moves in the
# increment form -- read u, q, c and write u, q (20 B); the recompute also
# stores a^n = L u^n + f^n (4 B), the adjoint reads it back (4 B); 68 B per
# point-step and shot over the three sweeps.  A temporally blocked kernel moves
# less, so this figure is reported as a rate only, never as a roofline fraction.
BYTES_PER_POINT_STEP = {"forward": 20.0, "recompute": 24.0, "adjoint": 24.0,
                        "forward_store": 24.0}
# Compulsory HBM bytes of the blocked schedule, the roofline's per-unit figures:
# per padded point, pair and launch the state u, q and the coefficient c are
# read once (12 B) and u, q written once (8 B); the adjoint also adds its
# launch's imaging partial into the FP64 sum (8 B read + 8 B write); per
# point-step the modes that keep a^n store it (4 B) and the adjoint reads it (4 B).
COMPULSORY_PER_POINT_LAUNCH = {"forward": 20.0, "recompute": 20.0, "adjoint": 36.0,
                               "forward_store": 20.0}
COMPULSORY_PER_POINT_STEP = {"forward": 0.0, "recompute": 4.0, "adjoint": 4.0,
                             "forward_store": 4.0}
# VALU issue peak: one wave64 VALU instruction per SIMD every 4 cycles (16 lanes),
# 256 CUs x 4 SIMDs x 2.4 GHz / 4 = 614.4 G wave-instructions per second.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
# Algorithmic flops per point-step: the fourth-order Laplacian with symmetric
# weights (4 pair sums, 1 centre product, 4 fused multiply-adds = 13), the
# increment update q' = g (q + c L u), u' = g u + q' (5); the adjoint adds the
# imaging product-sum z a (2).
FLOPS_PER_POINT_STEP = {"forward": 18.0, "recompute": 18.0, "adjoint": 20.0,
                        "forward_store": 18.0}
COUNTERS = os.path.join(ROOT, "profiles", "fd_pipe_c2_counters.json")
STEP_SOURCES = [os.path.join(ROOT, "paper_2310_13325_amd", "csrc", f)
                for f in ("fwi.hip", "fd_block.h", "fd_block_body.inc", "fd_pipe.h")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash() -> str:
    """Hash of the time-stepping kernel's sources (counters go stale with them)."""
    h = hashlib.sha256()
    for path in STEP_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_counters(configuration: dict):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel source in the same configuration (tile
    shape, stored steps, live pairs)."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("source_sha256_16") != source_hash() or c.get("configuration") != configuration:
        return None
    return c


def stream_rates(torch, mib=1024, reps=5):
    """What plain streaming kernels (torch's fill, copy and a + b) reach on this
    GPU, in GB/s of algorithmic bytes: a practical ceiling beside the published
    HBM peak."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    out = {}
    for name, fn, nbytes in (("fill", lambda: c.fill_(2.0), 4 * n),
                             ("copy", lambda: c.copy_(a), 8 * n),
                             ("add", lambda: torch.add(a, b, out=c), 12 * n)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del a, b, c
    torch.cuda.empty_cache()
    return out


def setup(prob, ctx, vb, synth, torch, npart):
    import numpy as np
    v, vbg = synth.true_model(prob)
    lo, hi = synth.prior_bounds(prob, v, vbg)
    parts = np.clip(synth.initial_particles(prob, lo, hi, npart), lo, hi)
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    grid = vb.Grid(nx=prob.nx, nz=prob.nz, nt=prob.nt, dx=prob.dx, dt=prob.dt,
                   vmax=float(np.float32(hi.max())), nb=prob.nb, sponge_alpha=prob.alpha)
    w = vb.vip_ricker(ctx, prob.nt, prob.dt, prob.f0)
    geom = vb.Geometry([prob.src_iz] * prob.ns, prob.src_ix, [prob.rec_iz] * prob.nr,
                       prob.rec_ix, w)
    clean = vb.vip_forward(ctx, grid, geom, f32(v[None]))[0]
    sigma = 0.02 * float(clean.abs().amax(dim=1).median())
    dobs = (clean + sigma * f32(synth.noise(prob))).contiguous()
    return dict(grid=grid, geom=geom, x=f32(parts), lo=f32(lo), hi=f32(hi), dobs=dobs,
                sigma=sigma, v_true=v, lo_np=lo, hi_np=hi, parts=parts)


def cpu_baseline(prob, S, ctx, vb, torch, workers, sched):
    """The FP64 oracle (a process per shot) on one particle of the workload,
    plus the GPU's error against it on the same inputs, the GPU run in the
    timed configuration (the context's tile, the timed memory schedule)."""
    import numpy as np
    from oracle import cpu_pool
    from oracle import fwi as ofwi
    grid = ofwi.Grid(nz=prob.nz, nx=prob.nx, nb=prob.nb, nt=prob.nt, dx=prob.dx, dz=prob.dx,
                     dt=prob.dt, alpha=prob.alpha)
    geom = ofwi.Geometry(src_iz=(prob.src_iz,) * prob.ns, src_ix=prob.src_ix,
                         rec_iz=(prob.rec_iz,) * prob.nr, rec_ix=prob.rec_ix, f0=prob.f0)
    v_true = np.float32(S["v_true"]).astype(np.float64)
    clean = cpu_pool.simulate(v_true, grid, geom, workers)
    sigma = 0.02 * float(np.median(np.abs(clean).max(axis=1)))
    from paper_2310_13325_amd import synth
    dobs = np.float32(clean + sigma * synth.noise(prob)).astype(np.float64)
    part = np.float32(S["parts"][:1]).astype(np.float64)
    t0 = time.perf_counter()
    lp_ref, g_ref = cpu_pool.grad_logpost(part, grid, geom, dobs, sigma, workers)
    wall = time.perf_counter() - t0
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    lp, g = vb.vip_grad_logpost(ctx, S["grid"], S["geom"], f32(part), f32(dobs), sigma,
                                ckpt_every=prob.ckpt_every, stored_steps=sched["stored_steps"],
                                live_pairs=sched["live_pairs"], ws_tag="err")
    g = g.cpu().numpy().astype(np.float64)
    err_g = float(np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref))
    err_lp = float(abs(lp.cpu().numpy()[0] - lp_ref[0]) / abs(lp_ref[0]))
    # one core: shot 0 of the same particle in this process, scaled to all shots
    geom1 = ofwi.Geometry(src_iz=(prob.src_iz,), src_ix=(prob.src_ix[0],),
                          rec_iz=(prob.rec_iz,) * prob.nr, rec_ix=prob.rec_ix, f0=prob.f0)
    t1 = time.perf_counter()
    ofwi.data_gradient(part[0], grid, geom1, dobs[:1], sigma)
    one_shot = time.perf_counter() - t1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    base = {"value": round(1.0 / wall, 5), "unit": "particle-gradients/s", "cores": workers,
            "kind": "oracle",
            "sample": f"1 particle x {prob.ns} shots of the workload, FP64 NumPy, one process "
                      f"per shot on {workers} host cores, {wall:.1f} s wall",
            "value_1core": round(1.0 / (one_shot * prob.ns), 5),
            "sample_1core": f"shot 0 of the same particle in one process ({one_shot:.1f} s), "
                            f"times {prob.ns} shots",
            "cpu_model": model}
    err = {"grad_rel_l2": err_g, "logpost_rel": err_lp,
           "against": "FP64 oracle, 1 particle, the timed tile and memory schedule"}
    return base, err


def advi_rates(prob, S, ctx, vb, torch, sched):
    """ADVI (section 2.2) on the same posterior in the unconstrained space of
    eq:transform, from N(0, I) as in section 4.1, one Monte Carlo sample per
    iteration (Table 1 counts one simulation per ADVI iteration) and eight:
    whole iterations per second (normals, sample, gradients, Adam step) for
    both families, and the HBM rate of the two full-rank kernels that stream
    the d(d+1)/2 entries of L (the sample reads 4 B per entry, the Adam step
    reads and writes L and two state arrays, 24 B per entry)."""
    from paper_2310_13325_amd import autotune
    prior = vb.Prior.transform(S["lo"], S["hi"])
    d = prob.d
    main_tile = ctx.tile_for(S["grid"])
    out = {"d": d, "prior": "uniform, transformed (eq:transform)", "rule": "adam",
           "eps": 1e-3}
    ev = lambda: torch.cuda.Event(enable_timing=True)
    for label, family, nsamp in (("full_rank_S1", vb.VIP_ADVI_FULL_RANK, 1),
                                 ("full_rank_S8", vb.VIP_ADVI_FULL_RANK, 8),
                                 ("mean_field_S1", vb.VIP_ADVI_MEAN_FIELD, 1)):
        # the gradient call has only nsamp x 10 pairs here: tune its tile and
        # memory schedule for that batch (untimed)
        th = torch.zeros(nsamp, prob.nz, prob.nx, device="cuda")
        lp = torch.empty(nsamp, dtype=torch.float64, device="cuda")
        gg = torch.empty_like(th)
        fn = lambda st, live: vb.vip_grad_logpost(
            ctx, S["grid"], S["geom"], th, S["dobs"], S["sigma"], ckpt_every=prob.ckpt_every,
            live_pairs=live, logpost=lp, grad=gg, stored_steps=st, prior=prior, ws_tag="advi")
        tile, stored, _, _ = autotune.tune_joint(ctx, fn, [(sched["stored_steps"], 0), (0, 0)])
        q = vb.Advi(d, family, kind=vb.VIP_OPT_ADAM)
        it = lambda k: vb.vip_advi_iteration(ctx, q, S["grid"], S["geom"], S["dobs"], S["sigma"],
                                             prior, nsamp, 1e-3, seed=2310, it=k,
                                             ckpt_every=prob.ckpt_every,
                                             stored_steps=stored, ws_tag="advi")
        it(0)
        torch.cuda.synchronize()
        reps = 5
        t = time.perf_counter()
        for k in range(reps):
            elbo = it(1 + k)
        torch.cuda.synchronize()
        rate = reps / (time.perf_counter() - t)
        out[label] = {"iterations_per_s": round(rate, 3),
                      "simulations_per_s": round(rate * nsamp, 3),
                      "tile": tile, "stored_steps": stored,
                      "elbo_last": float(elbo.item())}
        if label == "full_rank_S8":
            # the two full-rank kernels alone, HIP events on the context stream
            eta = vb.vip_philox_normals(ctx, nsamp * d, 7, 0).view(nsamp, d)
            g = 1e-3 * vb.vip_philox_normals(ctx, nsamp * d, 7, 1).view(nsamp, d)
            entries = d * (d + 1) / 2
            for kname, call, bpe in (
                    ("advi_sample_full", lambda: vb.vip_advi_sample(ctx, q, eta), 4.0),
                    ("advi_step_full_adam", lambda: vb.vip_advi_step(ctx, q, eta, g, 0.0), 24.0)):
                call()
                a, b = ev(), ev()
                n = 10
                a.record()
                for _ in range(n):
                    call()
                b.record()
                torch.cuda.synchronize()
                us = a.elapsed_time(b) * 1e3 / n
                gbs = bpe * entries / (us * 1e-6) / 1e9
                out[label][kname] = {"avg_launch_us": round(us, 1),
                                     "alg_bytes_per_launch": int(bpe * entries),
                                     "alg_GBps": round(gbs, 1),
                                     "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                                     "samples": nsamp}
        del q
        ctx._ws.pop("advi", None)
        torch.cuda.empty_cache()
    ctx.set_tile(main_tile)
    return out


def _timed(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps


def c1_rate(ctx, vb, synth, torch, configs):
    """c1: the plain SVGD-FWI loop, 8 particles x 4 shots on 64 x 64 cells,
    nt = 500: 20 iterations of the gradients plus an SVGD step (FP32 Gram,
    median bandwidth, clip)."""
    prob = configs.C1
    S1 = setup(prob, ctx, vb, synth, torch, prob.np)
    n, d = prob.np, prob.d
    # the tile shape the library picks for this small grid (32 pairs), not the
    # one tuned for the main workload
    main_tile = ctx.tile_for(S1["grid"])   # the context's setting (tuned or fixed)
    ctx.set_tile(-2)
    X = S1["x"].view(n, d)
    lp = torch.empty(n, dtype=torch.float64, device="cuda")
    g = torch.empty_like(S1["x"])
    eps = {}

    def run():
        for _ in range(configs.SVGD_STEPS_C1):
            vb.vip_grad_logpost(ctx, S1["grid"], S1["geom"], S1["x"], S1["dobs"], S1["sigma"],
                                ckpt_every=prob.ckpt_every, lo=S1["lo"], hi=S1["hi"],
                                logpost=lp, grad=g, ws_tag="c1")
            if "eps" not in eps:
                eps["eps"] = 10.0 / float(g.abs().max())
            vb.vip_svgd_step(ctx, X, g.view(n, d), eps["eps"], gram_prec=vb.VIP_GRAM_FP32,
                             lo=S1["lo"].view(-1), hi=S1["hi"].view(-1), ws_tag="c1svgd")

    sec = _timed(torch, run, 3)
    ctx._ws.pop("c1", None)
    ctx._ws.pop("c1svgd", None)
    steps = configs.SVGD_STEPS_C1
    tile = ctx.tile_for(S1["grid"], n * prob.ns)
    ctx.set_tile(main_tile)
    return {"workload": "c1: 64x64 at 10 m, nt=500, 4 shots, 64 receivers, 8 particles, "
                        f"{steps} SVGD iterations (gradients + FP32-Gram SVGD step)",
            "svgd_iterations_per_s": round(steps / sec, 1),
            "particle_gradients_per_s": round(steps * n / sec, 1), "tile": tile}


def c3_rate(ctx, vb, synth, torch, configs, autotune, fixed=None):
    """c3: 64 particles x 20 shots on 400 x 200 cells at 12.5 m, nt = 4000:
    particle-gradients/s with the tile and memory schedule (checkpoint
    interval 50, stored tail steps, live pairs) picked by the autotuner, or
    `fixed` = (tile, stored_steps, live_pairs)."""
    prob = configs.C3
    S3 = setup(prob, ctx, vb, synth, torch, prob.np)
    n = prob.np
    lp = torch.empty(n, dtype=torch.float64, device="cuda")
    g = torch.empty_like(S3["x"])
    fn = lambda st, live: vb.vip_grad_logpost(
        ctx, S3["grid"], S3["geom"], S3["x"], S3["dobs"], S3["sigma"], ckpt_every=prob.ckpt_every,
        lo=S3["lo"], hi=S3["hi"], logpost=lp, grad=g, stored_steps=st, live_pairs=live,
        ws_tag="c3")
    torch.cuda.empty_cache()
    if fixed is None:
        budget = int(torch.cuda.mem_get_info()[0] + ctx.workspace_bytes() - 8e9)
        cands = autotune.schedules(S3["grid"], S3["geom"], n, prob.ckpt_every, budget)
        tile, st, live, tm = autotune.tune_joint(ctx, fn, cands, tiles=[0, 2, 6])
    else:
        tile, st, live = fixed
        cands = [(st, live)]
        ctx.set_tile(tile)
    ctx.read_timing()
    ctx.set_timing(True)
    sec = _timed(torch, lambda: fn(st, live), 2)
    ctx.set_timing(False)
    timing = ctx.read_timing()
    ctx._ws.pop("c3", None)
    torch.cuda.empty_cache()
    npts = (prob.nx + 2 * prob.nb) * (prob.nz + 2 * prob.nb)
    modes = {k: {"launches": t["launches"],
                 "avg_launch_us": round(t["ms"] * 1e3 / t["launches"], 2)}
             for k, t in timing.items() if t["launches"]}
    return {"workload": "c3: 400x200 at 12.5 m + 20-cell sponge, nt=4000, dt=1 ms, 20 shots, "
                        "400 receivers, 10 Hz Ricker, 64 particles, checkpoints every 50 steps",
            "value": round(n / sec, 3), "unit": "particle-gradients/s",
            "ms_per_call": round(sec * 1e3, 1), "tile": tile, "stored_steps": st,
            "live_pairs": live, "schedules": [list(c) for c in cands], "modes": modes,
            # a streaming sweep (68 B per point-step and shot) at the HBM peak
            "streaming_ceiling_pg_per_s": round(
                HBM_PEAK_GBS * 1e9 / (68.0 * prob.ns * (prob.nt - 1) * npts), 2)}, S3


def c3_err(prob, S3, ctx, vb, torch, workers, sched):
    """The c3 gradient of one particle in the timed configuration against the
    FP64 C oracle (observed data from the oracle on the true model)."""
    import numpy as np
    from oracle import cref
    from oracle import fwi as ofwi
    from paper_2310_13325_amd import synth
    grid = ofwi.Grid(nz=prob.nz, nx=prob.nx, nb=prob.nb, nt=prob.nt, dx=prob.dx, dz=prob.dx,
                     dt=prob.dt, alpha=prob.alpha)
    geom = ofwi.Geometry(src_iz=(prob.src_iz,) * prob.ns, src_ix=prob.src_ix,
                         rec_iz=(prob.rec_iz,) * prob.nr, rec_ix=prob.rec_ix, f0=prob.f0)
    v_true = np.float32(S3["v_true"]).astype(np.float64)
    clean = cref.simulate(v_true, grid, geom, workers=workers)
    sigma = 0.02 * float(np.median(np.abs(clean).max(axis=1)))
    dobs = np.float32(clean + sigma * synth.noise(prob)).astype(np.float64)
    part = np.float32(S3["parts"][:1]).astype(np.float64)
    lp_ref, g_ref = cref.grad_logpost(part, grid, geom, dobs, sigma, workers=workers)
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    ctx.set_tile(sched["tile"])
    lp, g = vb.vip_grad_logpost(ctx, S3["grid"], S3["geom"], f32(part), f32(dobs), sigma,
                                ckpt_every=prob.ckpt_every, stored_steps=sched["stored_steps"],
                                live_pairs=sched["live_pairs"], ws_tag="c3err")
    g = g.cpu().numpy().astype(np.float64)
    ctx._ws.pop("c3err", None)
    return {"grad_rel_l2": float(np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)),
            "logpost_rel": float(abs(lp.cpu().numpy()[0] - lp_ref[0]) / abs(lp_ref[0])),
            "against": "FP64 C oracle, 1 particle, the timed tile and memory schedule"}


def c4_rates(ctx, vb, synth, torch, configs, autotune):
    """c4: three inversions of uneven size (96x96, 150x100, 256x128; nt 800,
    1200, 1600; 4, 6, 8 shots; 32 particles each) in merged launches against
    the three run one after the other, plus the batched sSVGD step (FP64
    Cholesky of each 32 x 32 kernel matrix)."""
    Ss = [setup(p, ctx, vb, synth, torch, p.np) for p in configs.C4]
    probs = [vb.Problem(S["grid"], S["geom"], S["x"], S["dobs"], S["sigma"], lo=S["lo"], hi=S["hi"])
             for S in Ss]
    key = autotune.key_for_batch(probs)
    tile = autotune.tune(ctx, lambda: vb.vip_grad_logpost_multi(ctx, probs, ckpt_every=50), key,
                         tiles=range(vb.lib().vip_tile_count()))
    batched = _timed(torch, lambda: vb.vip_grad_logpost_multi(ctx, probs, ckpt_every=50), 3)
    ctx.set_tile(-2)

    def one_by_one():
        for k, (S, p) in enumerate(zip(Ss, configs.C4)):
            vb.vip_grad_logpost(ctx, S["grid"], S["geom"], S["x"], S["dobs"], S["sigma"],
                                ckpt_every=50, lo=S["lo"], hi=S["hi"], logpost=probs[k].logpost,
                                grad=probs[k].grad, ws_tag=f"c4_{k}")

    separate = _timed(torch, one_by_one, 3)
    xs = [S["x"].view(p.np, p.d) for S, p in zip(Ss, configs.C4)]
    gs = [pr.grad.view(p.np, p.d) for pr, p in zip(probs, configs.C4)]
    eps = [10.0 / float(g.abs().max()) for g in gs]
    los = [S["lo"].view(-1) for S in Ss]
    his = [S["hi"].view(-1) for S in Ss]
    svgd = _timed(torch, lambda: vb.vip_ssvgd_step_multi(ctx, xs, gs, eps, seed=4, lo=los, hi=his,
                                                         gram_prec=vb.VIP_GRAM_FP32), 5)
    for k in range(3):
        ctx._ws.pop(f"c4_{k}", None)
    ctx._ws.pop("multi", None)
    ctx._ws.pop("svgd_multi", None)
    total = sum(p.np for p in configs.C4)
    return {"workload": "c4: 96x96 / 150x100 / 256x128 at 10 m, nt 800/1200/1600, 4/6/8 shots, "
                        "32 particles each",
            "batched_pg_per_s": round(total / batched, 1), "tile": tile,
            "one_by_one_pg_per_s": round(total / separate, 1),
            "batched_vs_one_by_one": round(separate / batched, 3),
            "ssvgd_multi_steps_per_s": round(1.0 / svgd, 1)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--particles", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-c5", action="store_true")
    ap.add_argument("--no-minibatch", action="store_true")
    ap.add_argument("--no-advi", action="store_true")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the c1, c3 and c4 workload rates")
    ap.add_argument("--workloads", default="c1,c4,c3",
                    help="which of the c1, c3, c4 workload rates to run (comma list)")
    ap.add_argument("--c3-schedule", default=None, metavar="TILE,STORED,LIVE",
                    help="fixed c3 tile and memory schedule (no tuning)")
    ap.add_argument("--graph", action="store_true", help="replay the gradient through a hipGraph")
    ap.add_argument("--tile", type=int, default=None, help="fixed tile shape (no tile tuning)")
    ap.add_argument("--stored-steps", type=int, default=None,
                    help="fixed stored tail steps (no schedule tuning)")
    ap.add_argument("--live-pairs", type=int, default=0)
    ap.add_argument("--no-tune", action="store_true",
                    help="automatic tile, every segment recomputed, all pairs live")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}); run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2310_13325_amd import autotune
    from paper_2310_13325_amd import binding as vb
    from paper_2310_13325_amd import configs, synth

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 4, "launches": 3}))
        return

    prob = configs.C2
    npart = args.particles or prob.np
    ctx = vb.Context(0, graph_mode=args.graph)
    log(f"setup: {prob.nx}x{prob.nz}, nt={prob.nt}, {prob.ns} shots, {npart} particles")
    S = setup(prob, ctx, vb, synth, torch, npart)
    n, d = npart, prob.d
    X = S["x"].view(n, d)
    lo, hi = S["lo"].view(-1), S["hi"].view(-1)
    logpost = torch.empty(n, dtype=torch.float64, device="cuda")
    grad = torch.empty_like(S["x"])
    G = grad.view(n, d)
    eps_holder = {}

    # Untimed set-up: the autotuner times every tile shape under every memory
    # schedule (stored tail steps, live pairs) that fits the free HBM and keeps
    # the fastest pair; --tile / --stored-steps fix either, --no-tune both.
    sched = {"stored_steps": 0, "live_pairs": 0}

    def grad_call(stored, live):
        vb.vip_grad_logpost(ctx, S["grid"], S["geom"], S["x"], S["dobs"], S["sigma"],
                            ckpt_every=prob.ckpt_every, lo=S["lo"], hi=S["hi"],
                            logpost=logpost, grad=grad, stored_steps=stored, live_pairs=live)

    if args.tile is not None:
        ctx.set_tile(args.tile)
    if args.stored_steps is not None:
        sched = {"stored_steps": args.stored_steps, "live_pairs": args.live_pairs}
    if not args.no_tune and (args.tile is None or args.stored_steps is None):
        torch.cuda.empty_cache()
        free = torch.cuda.mem_get_info()[0] + ctx.workspace_bytes()
        budget = int(free - 8e9)
        cands = ([(sched["stored_steps"], sched["live_pairs"])] if args.stored_steps is not None
                 else autotune.schedules(S["grid"], S["geom"], n, prob.ckpt_every, budget))
        tiles = [args.tile] if args.tile is not None else None
        tile, st, live, tm = autotune.tune_joint(ctx, grad_call, cands, tiles=tiles)
        sched = {"stored_steps": st, "live_pairs": live}
        log(f"autotuned tile {tile}, memory schedule {sched} over {len(tm)} candidates "
            f"(schedules {cands})")

    def step(i):
        grad_call(sched["stored_steps"], sched["live_pairs"])
        if "eps" not in eps_holder:
            # step size giving updates of about 10 m/s (fixed after the first gradient)
            eps_holder["eps"] = 10.0 / float(G.abs().max())
        vb.vip_ssvgd_step(ctx, X, G, eps_holder["eps"], xi=None, seed=231013325, stream=i,
                          gram_prec=vb.VIP_GRAM_BF16, lo=lo, hi=hi)

    for i in range(args.warmup):
        step(i)
        log(f"warmup step {i} done")
    torch.cuda.synchronize()
    ctx.read_timing()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.set_timing(False)
    timing = ctx.read_timing()
    timed_calls = args.steps   # gradient calls the per-launch timing covers
    if args.graph and not any(t["launches"] for t in timing.values()):
        # graph replays carry no per-launch events: time the step kernel on one
        # eager gradient call after the timed region
        ctx.set_graph_mode(False)
        ctx.set_timing(True)
        grad_call(sched["stored_steps"], sched["live_pairs"])
        torch.cuda.synchronize()
        ctx.set_timing(False)
        timing = ctx.read_timing()
        timed_calls = 1
        ctx.set_graph_mode(True)
    flags = ctx.poll(ctx.workspace("grad", 0)) | ctx.poll(ctx.workspace("svgd", 0))
    log(f"timed {args.steps} steps in {elapsed:.3f} s; device flags {flags}")
    if not bool(torch.isfinite(X).all()):
        raise RuntimeError("non-finite particles after the timed steps")

    value = args.steps * n / elapsed
    tile = ctx.tile_for(S["grid"])
    if tile >= 0:
        sh = vb.tile_shape(tile)
        kname = (f"{'fd_pipe (persistent, ' if sh['persistent'] else 'fd_block ('}"
                 f"temporally blocked, {sh['ex']}x{sh['ez']} extended tile, "
                 f"up to {sh['tmax']} steps per launch)")
    else:
        kname = "fd_step (one step per launch)"
    # pairs each launch advances: the live pairs of a chunk (equal chunks but
    # possibly a shorter last one; every chunk runs the same launches)
    pairs = n * prob.ns
    live = sched["live_pairs"] or pairs
    nchunks = -(-pairs // live)
    npts = (prob.nx + 2 * prob.nb) * (prob.nz + 2 * prob.nb)
    kinds = {}
    for k, t in timing.items():
        if t["launches"]:
            per_launch_s = t["ms"] * 1e-3 / t["launches"]
            ps = t["point_steps"] / t["launches"]
            # pair-points per launch, averaged over the chunks (each chunk runs
            # the same number of launches)
            pl = pairs * npts / nchunks
            comp = COMPULSORY_PER_POINT_LAUNCH[k] * pl + COMPULSORY_PER_POINT_STEP[k] * ps
            kinds[k] = {"launches": t["launches"], "avg_launch_us": round(per_launch_s * 1e6, 2),
                        "point_steps_per_launch": ps,
                        "compulsory_bytes_per_launch": int(comp),
                        "compulsory_GBps": round(comp / per_launch_s / 1e9, 1),
                        "streaming_equivalent_GBps": round(
                            BYTES_PER_POINT_STEP[k] * ps / per_launch_s / 1e9, 1),
                        "alg_TFLOPs": round(FLOPS_PER_POINT_STEP[k] * ps / per_launch_s / 1e12, 3),
                        "share_of_step": round(t["ms"] / 1e3 / (elapsed / args.steps * timed_calls), 3)}
    dom = max(kinds, key=lambda k: kinds[k]["share_of_step"])
    ach = kinds[dom]["compulsory_GBps"]
    counters = traffic_from_counters({"tile": tile, "stored_steps": sched["stored_steps"],
                                      "live_pairs": sched["live_pairs"]})
    tr = None if counters is None else counters.get("traffic_bytes_per_launch", {}).get(dom)
    vi = None if counters is None else counters.get("valu_instr_per_launch", {}).get(dom)
    launch_s = kinds[dom]["avg_launch_us"] * 1e-6
    meas = None if tr is None else round(tr / launch_s / 1e9, 1)
    roofline = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": tr,
                "bytes_model": "compulsory bytes of the blocked schedule per launch: "
                               "(u, q, c read + u, q written: 20 B; adjoint +16 B FP64 imaging "
                               "read-modify-write) per padded point and pair, plus 4 B of a^n "
                               "per point-step",
                # counter-measured HBM bytes per launch over the live launch time
                "measured_GBps": meas,
                # plain streaming kernels on the same GPU, for scale
                "stream_reference_GBps": stream_rates(torch),
                "measured_frac": None if meas is None else round(meas / HBM_PEAK_GBS, 4),
                "kernel": f"{kname}, {dom} mode", "modes": kinds,
                # VALU issue rate from the counted wave instructions (SQ_INSTS_VALU)
                "valu": None if vi is None else {
                    "achieved": round(vi / launch_s / 1e9, 1), "peak": VALU_ISSUE_PEAK / 1e9,
                    "unit": "G wave-instr/s", "frac": round(vi / launch_s / VALU_ISSUE_PEAK, 4)},
                "alu": {"achieved": kinds[dom]["alg_TFLOPs"], "peak": ALU_PEAK_TFLOPS,
                        "unit": "TFLOP/s",
                        "frac": round(kinds[dom]["alg_TFLOPs"] / ALU_PEAK_TFLOPS, 4),
                        "frac_of_published": round(kinds[dom]["alg_TFLOPs"] / ALU_PUBLISHED_TFLOPS, 4)},
                # particle-gradients/s of a streaming implementation at the HBM
                # peak: forward, recompute and adjoint sweeps (20 + 24 + 24 B per
                # point-step and shot), or forward-with-store and adjoint (24 + 24)
                "streaming_ceiling_pg_per_s": {
                    label: round(HBM_PEAK_GBS * 1e9 / (b * prob.ns * (prob.nt - 1)
                                                       * (prob.nx + 2 * prob.nb)
                                                       * (prob.nz + 2 * prob.nb)), 1)
                    for label, b in (("recompute", 68.0), ("stored", 48.0))}}

    extra = {}
    if not args.no_minibatch:
        # Section 2.4's minibatch gradients: b of the 10 shots per iteration,
        # drawn uniformly without replacement, each an unbiased estimate
        ctx._ws.pop("grad", None)
        torch.cuda.empty_cache()
        b = 2
        subsets = synth.minibatch_shots(prob.seed, prob.ns, b, 6)
        mb = lambda shots: vb.vip_grad_logpost_minibatch(
            ctx, S["grid"], S["geom"], S["x"], S["dobs"], S["sigma"], shots,
            ckpt_every=prob.ckpt_every, lo=S["lo"], hi=S["hi"], logpost=logpost, grad=grad,
            stored_steps=sched["stored_steps"], ws_tag="minibatch")
        mb(subsets[0])
        torch.cuda.synchronize()
        t = time.perf_counter()
        for shots in subsets[1:]:
            mb(shots)
        torch.cuda.synchronize()
        rate = (len(subsets) - 1) * n / (time.perf_counter() - t)
        extra["minibatch"] = {"shots_per_batch": b, "of_shots": prob.ns, "value": round(rate, 2),
                              "unit": "particle-gradient estimates/s",
                              "vs_full": round(rate / value, 2)}
        ctx._ws.pop("minibatch", None)
        log(f"minibatch {b} of {prob.ns} shots: {rate:.1f} estimates/s")
    if not args.no_advi:
        extra["advi"] = advi_rates(prob, S, ctx, vb, torch, sched)
        log(f"advi: {extra['advi']}")
    main_tile = ctx.tile_for(S["grid"])
    S3 = sched3 = None
    if not args.no_workloads:
        ctx._ws.pop("grad", None)
        torch.cuda.empty_cache()
        work = {}
        which = [w.strip() for w in args.workloads.split(",") if w.strip()]
        if "c1" in which:
            work["c1"] = c1_rate(ctx, vb, synth, torch, configs)
            log(f"c1: {work['c1']}")
        if "c4" in which:
            work["c4"] = c4_rates(ctx, vb, synth, torch, configs, autotune)
            log(f"c4: {work['c4']}")
        if "c3" in which:
            fixed = (None if args.c3_schedule is None
                     else tuple(int(v) for v in args.c3_schedule.split(",")))
            work["c3"], S3 = c3_rate(ctx, vb, synth, torch, configs, autotune, fixed)
            sched3 = {"tile": work["c3"]["tile"], "stored_steps": work["c3"]["stored_steps"],
                      "live_pairs": work["c3"]["live_pairs"]}
            log(f"c3: {work['c3']}")
        extra["workloads"] = work
        ctx.set_tile(main_tile)
    if not args.no_plain:
        x1 = S["x"][:1].contiguous()
        vb.vip_grad_logpost_plain(ctx, S["grid"], S["geom"], x1, S["dobs"], S["sigma"],
                                  lo=S["lo"], hi=S["hi"])
        torch.cuda.synchronize()
        t = time.perf_counter()
        vb.vip_grad_logpost_plain(ctx, S["grid"], S["geom"], x1, S["dobs"], S["sigma"],
                                  lo=S["lo"], hi=S["hi"])
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        extra["plain_path"] = {"value": round(1.0 / tp, 4), "unit": "particle-gradients/s",
                               "speedup": round(value * tp, 2),
                               "what": "one pair at a time, unfused per-step launches"}
        log(f"plain path: {1.0 / tp:.3f} particle-gradients/s")
    if not args.no_c5:
        case = configs.C5
        # the c5 inputs: the c2 model perturbed by smoothed seeded fields, and
        # gradients pulling towards it (the parity test's generator)
        Xn, Gn = synth.svgd_precision_case(case, S["v_true"])
        Xc = torch.as_tensor(Xn, dtype=torch.float32, device="cuda")
        Gc = torch.as_tensor(Gn, dtype=torch.float32, device="cuda")
        del Xn, Gn
        svgd = {}
        reps = 20   # about 25 ms per path: long enough for stable clocks and timing
        for name, prec in (("bf16_gram", vb.VIP_GRAM_BF16), ("fp32_gram", vb.VIP_GRAM_FP32)):
            Xw = Xc.clone()
            for _ in range(3):
                vb.vip_svgd_step(ctx, Xw, Gc, case.eps, gram_prec=prec, ws_tag="c5")
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                vb.vip_svgd_step(ctx, Xw, Gc, case.eps, gram_prec=prec, ws_tag="c5")
            torch.cuda.synchronize()
            svgd[name] = round(reps / (time.perf_counter() - t), 2)
        # the diagonal matrix-valued kernel (Q = 1 / per-coordinate variance), BF16 Gram
        Xw = Xc.clone()
        diag = lambda: vb.vip_svgd_step_ex(ctx, Xw, Gc, case.eps, kernel=vb.VIP_KERNEL_DIAG_VAR,
                                           gram_prec=vb.VIP_GRAM_BF16, ws_tag="c5")
        for _ in range(3):
            diag()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            diag()
        torch.cuda.synchronize()
        svgd["bf16_gram_diag_kernel"] = round(reps / (time.perf_counter() - t), 2)
        # sSVGD at the paper's FWI ensemble size (600) and at n = 2048: the
        # noise needs the FP64 Cholesky of K/n, blocked over the GPU beyond 128
        for nn in (600, 2048):
            Xs, Gs = Xc[:nn].clone(), Gc[:nn].contiguous()
            call = lambda k: vb.vip_ssvgd_step(ctx, Xs, Gs, case.eps, seed=5, stream=k,
                                               gram_prec=vb.VIP_GRAM_BF16, ws_tag="c5s")
            for k in range(2):
                call(k)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for k in range(10):
                call(2 + k)
            torch.cuda.synchronize()
            svgd[f"ssvgd_bf16_gram_n{nn}"] = round(10 / (time.perf_counter() - t), 2)
            del Xs, Gs
        ctx._ws.pop("c5s", None)
        # Matrix-core work of one BF16-path step against the dense BF16 peak,
        # two ways: algorithmic -- the upper Gram (the 136 upper 128 x 128
        # blocks of 256, 2 n^2 d x 136/256) and one product K B (2 n^2 d); and
        # executed -- the Gram kernel computes whole upper 256 x 256 blocks
        # (36 of 64 at n = 2048) and the update runs the product as two BF16
        # products (K times the two halves of the split B)
        nn_d = 2.0 * case.n * case.n * case.d
        nb = (case.n + 127) // 128
        gram = nn_d * (nb * (nb + 1) / 2) / nb ** 2
        nb2 = (case.n + 255) // 256
        gram_run = nn_d * (nb2 * (nb2 + 1) / 2) / nb2 ** 2
        alg, executed = gram + nn_d, gram_run + 2.0 * nn_d
        rate = svgd["bf16_gram"]
        svgd["bf16_path_matrix_core"] = {
            "algorithmic_flops_per_step": alg, "algorithmic_TFLOPs": round(alg * rate / 1e12, 1),
            "algorithmic_frac": round(alg * rate / 2.5e15, 4),
            "executed_flops_per_step": executed,
            "executed_TFLOPs": round(executed * rate / 1e12, 1),
            "executed_frac": round(executed * rate / 2.5e15, 4), "peak_TFLOPs": 2500.0,
            "profile": "profiles/svgd_c5.md (per-kernel MFMA busy from counters)"}
        extra["svgd_steps_per_s"] = {"n": case.n, "d": case.d, **svgd}
        log(f"svgd c5: {svgd}")
        ctx._ws.pop("c5", None)

    cpu = None
    err = None
    if not args.no_cpu_baseline:
        from oracle import cpu_pool
        workers = min(cpu_pool.default_workers(), prob.ns)
        log(f"cpu baseline on {workers} cores")
        cpu, err = cpu_baseline(prob, S, ctx, vb, torch, workers, sched)
        if S3 is not None:
            extra["workloads"]["c3"]["err"] = c3_err(configs.C3, S3, ctx, vb, torch,
                                                     cpu_pool.default_workers(), sched3)
            ctx.set_tile(main_tile)
            log(f"c3 err: {extra['workloads']['c3']['err']}")

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "particle-gradients/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": "c2: FP32 batched gradients + sSVGD step; 200x120 grid at 20 m "
                               "+ 20-cell sponge, nt=2000, dt=2 ms, 10 shots, 200 receivers, "
                               "8 Hz Ricker, 128 particles; memory schedule as tuned "
                               "(stored_steps a^n kept by the forward sweep, the rest "
                               "checkpointed every 50 steps)",
                   "particles": n, "pairs_per_step": n * prob.ns, "graph": args.graph,
                   "gram": "bf16", "parallelism": "1 GPU", "tile": ctx.tile_for(S["grid"]),
                   "stored_steps": sched["stored_steps"], "live_pairs": sched["live_pairs"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "err": err,
        **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
