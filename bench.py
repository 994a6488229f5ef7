#!/usr/bin/env python3
"""Benchmark: D-Landweber under AR boundary conditions on one MI355X.

A step is one pass of the whole hot path over the 1024x1024 workload:
residual r = g - A x (AR blur, FP64 norm partials), y = A' r (reblur),
c = T~ y along rows, the fused column pass T~ / filter d / T, and the row
pass T fused with x += tau w, i.e. one preconditioned Landweber iteration
including its per-iteration FP64 residual norm.  The timed region runs
exactly K steps, as consecutive runs of at most 100 iterations from
x_0 = 0, with all inputs resident on the GPU; the per-iteration norms are
copied to the host once per run (inside the timed region).  The timed runs
use a Tikhonov parameter at which the iteration is stable (0.2); the
workload's named 5e-3 makes it diverge and is reported under "quality".

Prints one JSON line: throughput, the roofline of the dominant kernel and
of the whole step (algorithmic bytes), per-kernel rooflines, restoration
quality and GPU time to the best relative error (plain, preconditioned,
learned), the batched workload, the learned-vs-plain sweep comparison, the
2048^2 precision variant, and the FP64 oracle timed on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f32|f32x]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

METRIC = "Mpixel-iters/s at 1024² FP32 + GPU time to best rel. error, learned vs plain"
WORKLOAD = "ar1024_f32_motion15"
ITERS = 100   # iterations of one run of the workload (its configuration)

# MI355X published peaks used for the roofline (dense, per GPU)
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6   # 256 CUs x 64 FP64 FMA lanes/clk x 2 flop x 2.4 GHz
FP32_VECTOR_TFLOPS = 157.3  # 256 CUs x 128 FP32 FMA lanes/clk x 2 flop x 2.4 GHz

# Algorithmic HBM bytes per pixel and iteration (FP32 images), by phase:
# r = g - A x reads x, g and writes r; y = A' r reads r, writes y; the
# transforms with the filter and the update read y, d, x and write x,
# which the three transform passes own as y (row pass of T~), d (column
# pass) and x read + written (row pass of T + update).  Intermediates
# between the passes and halo re-reads are implementation traffic.
ALG_BYTES = {"residual": 12, "reblur": 8, "row_fwd": 4, "col": 4, "row_inv": 8}
STEP_BYTES = sum(ALG_BYTES.values())   # 36 B per pixel-iteration


def step_flops(n1, n2, taps):
    """Algorithmic flops per pixel-iteration: the blur and the reblur (2 P
    each, P = PSF taps), the forward and inverse 2-D AR transforms at the
    ideal FFT count 5 log2(2 (m - 1)) per axis and direction (m the axis
    length: the DST-I of the interior through a length-2(m-1) real FFT),
    and the residual, filter and update (3).  A fixed convention, like the
    36 B: the radix-31/11/3 stages and the packing cost more than this."""
    ft = 2 * 5 * math.log2(2 * (n1 - 1)) + 2 * 5 * math.log2(2 * (n2 - 1))
    return 4 * taps + ft + 3
STABLE_ALPHA = 0.2          # 1024^2 motion PSF: I - D A'A has spectral radius ~1
BATCH_STABLE_ALPHA = 0.5    # every batched Gaussian PSF: spectral radius <= 1
PLAIN_CAP = 3000            # iteration cap of the unpreconditioned run to its best RRE


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000,
                    help="timed iterations, run as consecutive runs of at most 100 from x = 0")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f32x"],
                    help="f32: FP32 images and arithmetic (meets the 1e-5 one-step bound for "
                         "alpha >= 0.05); f32x: FP32 images, FP64 arithmetic (any alpha)")
    ap.add_argument("--alpha", type=float, default=STABLE_ALPHA,
                    help="Tikhonov parameter of the timed runs (the named 5e-3 diverges)")
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--no-tune", action="store_true", help="skip the plan autotuner")
    ap.add_argument("--tuning", default=None,
                    help="JSON object of launch settings (the keys of the output's 'tuning') "
                         "to set instead of autotuning, e.g. to repeat a run's choice under a "
                         "profiler, whose per-dispatch overhead would mislead the autotuner")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-bc", action="store_true",
                    help="skip the Reflective / Periodic and direct-solve legs")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the 2048^2 BF16x3 precision-variant leg")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one torch copy of 256 MiB (reference for HBM counters)")
    ap.add_argument("--learned-images", type=int, default=64,
                    help="images of the learned-vs-plain leg (0 skips it)")
    return ap.parse_args()


def make_inputs(torch, P, dt):
    import synth
    F, H, E, p = synth.workload(WORKLOAD)
    n = p["n"]
    tdt = torch.float32
    f = torch.from_numpy(F).to("cuda:0", tdt)
    e = torch.from_numpy(E).to("cuda:0", tdt)
    plan = P.Plan(n, n, H, dtype=dt)
    b = torch.empty_like(f)
    plan.ar_blur_apply(f, b)                       # noise-free data A f on the GPU
    g = b + (p["nu"] * torch.linalg.vector_norm(b.double()) /
             torch.linalg.vector_norm(e.double())).float() * e
    torch.cuda.synchronize()
    return plan, f, g, F, H, E, p


def source_digest():
    """SHA-256 over the library's HIP sources (identifies the kernels that
    a set of hardware counters was taken on)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1211_0393_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(dtype):
    """HBM bytes per launch from the committed hardware-counter summary
    (profiles/traffic.json: FETCH_SIZE and WRITE_SIZE per dispatch, scaled
    by the same counters of a plain copy of known size), keyed by phase
    name; empty when the kernels changed since the counters were taken."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return {}
    if t.get("source_sha256") != source_digest() or t.get("dtype") != dtype:
        return {}
    return {k: v["hbm_bytes_per_launch"] for k, v in t.get("phases", {}).items()}


def diverged(res):
    """A run diverged when a residual norm is not finite or some later
    residual exceeds the initial one ||g - A x_0||."""
    if res is None or len(res) == 0:
        return False
    res = np.asarray(res)
    return bool(not np.all(np.isfinite(res)) or (len(res) > 1 and np.max(res[1:]) > res[0]))


def finite_min(v):
    if v is None:
        return None
    v = np.asarray(v)
    v = v[np.isfinite(v)]
    return float(v.min()) if v.size else None


def _oracle_rate(G, H, d, iters, workers=1):
    """Mpixel-iters/s of `iters` FP64 oracle D-Landweber steps (after one
    warm-up step) with scipy.fft using `workers` threads."""
    import scipy.fft
    import oracle as O
    X = np.zeros_like(G)
    with scipy.fft.set_workers(workers):
        X, _ = O.landweber_step(X, G, H, d=d)          # warm-up
        t0 = time.perf_counter()
        for _ in range(iters):
            X, _ = O.landweber_step(X, G, H, d=d)
        dt = time.perf_counter() - t0
    return G.size * iters / dt / 1e6, dt


def _oracle_batch_worker(args):
    i, iters = args
    import oracle as O
    import synth
    F, H, E, prm = synth.batch_problem(i)
    G = O.observe(F, H, E, prm["nu"])
    d = O.tikhonov(O.eigenvalues(H, *G.shape), BATCH_STABLE_ALPHA)
    X = np.zeros_like(G)
    t0 = time.perf_counter()
    for _ in range(iters):
        X, _ = O.landweber_step(X, G, H, d=d)
    return G.size * iters, time.perf_counter() - t0


def cpu_baseline(F, H, E, p, iters):
    """The FP64 oracle (as written, untuned) on this host, on bounded samples
    of the workloads: the 1024^2 workload single-threaded (the reported
    value) and with scipy.fft on every core (numpy's elementwise work stays
    on one thread); the 64^2 FP64 workload; one 512^2 batched problem on one
    core, and the batched workload's problems in a process pool over every
    core (aggregate throughput).  In Mpixel-iters/s."""
    import multiprocessing as mp
    import oracle as O
    import synth
    cores = os.cpu_count() or 1
    G = O.observe(F, H, E, p["nu"])
    d = O.tikhonov(O.eigenvalues(H, *G.shape), p["alpha"])
    v1, t1 = _oracle_rate(G, H, d, iters, workers=1)
    vall, tall = _oracle_rate(G, H, d, iters, workers=cores)
    F1, H1, E1, p1 = synth.workload("ar64_f64_gauss9")
    G1 = O.observe(F1, H1, E1, p1["nu"])
    d1 = O.tikhonov(O.eigenvalues(H1, *G1.shape), p1["alpha"])
    vc1, tc1 = _oracle_rate(G1, H1, d1, p1["iters"], workers=1)
    i512 = next(i for i in range(256) if synth.batch_problem(i)[3]["n"] == 512)
    px, t512 = _oracle_batch_worker((i512, iters))
    v512 = px / t512 / 1e6
    nproc = min(cores, 16)
    with mp.get_context("spawn").Pool(nproc) as pool:
        res = pool.map(_oracle_batch_worker, [(i, 3) for i in range(nproc)])
    tpool = max(r[1] for r in res)          # the workers run concurrently
    vpool = sum(r[0] for r in res) / tpool / 1e6
    modes = [
        {"workload": "1024x1024 15x15 motion PSF, D-Landweber", "threads": 1,
         "value": round(v1, 4), "seconds": round(t1, 2), "iterations": iters},
        {"workload": "1024x1024 15x15 motion PSF, D-Landweber", "threads": cores,
         "value": round(vall, 4), "seconds": round(tall, 2), "iterations": iters,
         "note": "scipy.fft workers = cores; elementwise numpy work single-threaded"},
        {"workload": "64x64 9x9 shifted Gaussian, FP64, D-Landweber", "threads": 1,
         "value": round(vc1, 4), "seconds": round(tc1, 2), "iterations": p1["iters"]},
        {"workload": "one 512x512 batched problem (Gaussian PSF)", "threads": 1,
         "value": round(v512, 4), "seconds": round(t512, 2), "iterations": iters},
        {"workload": f"{nproc} batched problems (n 128..512), one per process", "threads": nproc,
         "value": round(vpool, 4), "seconds": round(tpool, 2), "iterations": 3,
         "note": "aggregate pixel-iterations over the slowest worker's iteration time"},
    ]
    return {"value": v1, "unit": "Mpixel-iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} FP64 D-Landweber iterations of the 1024x1024 15x15-PSF workload "
                      f"after 1 warm-up ({t1:.1f} s); numpy/scipy on one thread "
                      f"(host os.cpu_count()={cores}); other modes and sizes in 'modes'",
            "modes": modes}


def bench_batch(torch, P, iters, count=256, alpha=BATCH_STABLE_ALPHA):
    """The batched workload: `count` problems (n in {128,...,512}, own
    Gaussian PSF 7..21 and noise level, FP32), `iters` preconditioned
    iterations in one graph launch, after a warm-up call that captures the
    graph.  Inputs are resident on the GPU.  The Tikhonov parameter is the
    smallest of 0.05, 0.1, 0.2, 0.3, 0.5 at which I - D A'A has spectral
    radius <= 1 for every PSF of the family (oracle power iteration); the
    value is reported only when every problem's run is finite and its
    residual never exceeds the initial one."""
    import synth
    plans, gs, xs = [], [], []
    px = 0
    for i in range(count):
        F, H, E, prm = synth.batch_problem(i)
        n = prm["n"]
        pl = P.Plan(n, n, H, dtype="f32")
        pl.ar_precond_set(P.AR_FILTER_TIKHONOV, alpha)
        f = torch.from_numpy(F).to("cuda:0", torch.float32)
        e = torch.from_numpy(E).to("cuda:0", torch.float32)
        b = torch.empty_like(f)
        pl.ar_blur_apply(f, b)
        g = b + (prm["nu"] * torch.linalg.vector_norm(b.double()) /
                 torch.linalg.vector_norm(e.double())).float() * e
        plans.append(pl)
        gs.append(g)
        xs.append(torch.zeros_like(g))
        px += n * n
    batch = P.Batch(plans)
    tuned = batch.ar_batch_autotune()
    batch.ar_batch_iterate(gs, xs, iters, want_resnorm=True)   # warm-up: captures the graph
    for x in xs:
        x.zero_()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    rc, res, _, _ = batch.ar_batch_iterate(gs, xs, iters, want_resnorm=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t = max(wall, ev0.elapsed_time(ev1) / 1e3)
    bad = sum(diverged(res[i]) for i in range(count))
    valid = rc == 0 and bad == 0
    out = {"workload": f"{count} problems, n in {{128,192,256,384,512}} (seed 404 + i), "
                       f"Gaussian PSFs 7..21, noise 0.1%..2%, Tikhonov alpha {alpha}, FP32, "
                       f"{iters} D-Landweber iterations in one graph launch",
           "value": round(px * iters / t / 1e6, 1) if valid else None, "unit": "Mpixel-iters/s",
           "measured_rate": round(px * iters / t / 1e6, 1),
           "valid": valid, "alpha": alpha,
           "pixels_per_iteration": px, "seconds": round(t, 5),
           "us_per_batch_iteration": round(t / iters * 1e6, 2),
           "status": rc, "autotuned_precond_us": round(tuned, 2),
           "diverged_problems": int(bad)}
    batch.close()
    for pl in plans:
        pl.close()
    return out


def bench_stable(torch, P, plan, f, g, net_path, iters=ITERS):
    """GPU time to the best relative error on the 1024^2 workload at a
    stable Tikhonov parameter (the named 5e-3 diverges): plain Landweber
    (D = I) run to PLAIN_CAP iterations, D-Landweber with Tikhonov
    STABLE_ALPHA, and the learned filter (features + network + gains
    filter, then D-Landweber), `iters` iterations each.  The time to best
    is the run's measured time per iteration times its best iteration, plus
    the filter set-up; reached_plain_best_at: the first iteration whose RRE
    is within 2% of the plain run's best (None if never)."""
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def run(k, precondition, setup=None):
        x = torch.zeros_like(g)
        torch.cuda.synchronize()
        ev[0].record(stream)
        if setup is not None:
            setup()
        ev[1].record(stream)
        rc, res, rre, best = plan.ar_deblur_iterate(g, x, k, precondition=precondition,
                                                    f_true=f, want_resnorm=True, want_rre=True)
        ev[2].record(stream)
        torch.cuda.synchronize()
        t_set = ev[0].elapsed_time(ev[1]) / 1e3
        t_it = ev[1].elapsed_time(ev[2]) / 1e3 / k
        return rc, res, rre, best, t_set, t_it

    def summary(rc, res, rre, best, t_set, t_it, ref=None):
        o = {"status": rc, "best_it": best, "best_rre": finite_min(rre),
             "us_per_iteration": round(t_it * 1e6, 2),
             "gpu_s_to_best": round(t_set + t_it * best, 6), "diverged": diverged(res)}
        if ref is not None:
            hit = np.nonzero(np.isfinite(rre) & (rre <= 1.02 * ref))[0]
            o["reached_plain_best_at"] = int(hit[0]) + 1 if hit.size else None
            o["gpu_s_to_plain_best"] = (round(t_set + t_it * (hit[0] + 1), 6)
                                        if hit.size else None)
        return o

    plain = summary(*run(PLAIN_CAP, False))
    ref = plain["best_rre"]
    pre = summary(*run(iters, True, lambda: plan.ar_precond_set(P.AR_FILTER_TIKHONOV,
                                                                STABLE_ALPHA)), ref=ref)
    out = {"workload": "1024x1024 motion-PSF workload (as the timed run), stable Tikhonov alpha",
           "alpha": STABLE_ALPHA, "plain_cap": PLAIN_CAP, "plain": plain,
           "preconditioned": pre}
    if net_path is not None:
        from paper_1211_0393_amd import learned as LR
        net = P.FNet(path=net_path)
        out["learned"] = summary(*run(iters, True, lambda: LR.apply_learned(net, plan, g)),
                                 ref=ref)
        net.close()
    if pre["best_it"]:
        out["iteration_ratio_plain_vs_preconditioned"] = round(plain["best_it"] /
                                                               pre["best_it"], 2)
    return out


def bench_learned(torch, P, images, iters):
    """GPU time to the best relative error, learned filter vs the plain
    method, on `images` problems at 1024^2 (PSFs 15..31 from three
    non-symmetric families, seeds 6,000,000 + i, noise 0.1%..2%).
    Plain: the whole 32-filter sweep (16 Tikhonov, 16 threshold
    parameters), `iters` iterations each, gives RRE* = its best RRE.
    Learned: features + network + gains filter + the iterations until
    RRE <= 1.02 RRE* (or its whole run when it never gets there).  Times
    are GPU event times on the current stream."""
    import synth
    from paper_1211_0393_amd import learned as LR
    try:
        params = LR.load_params()
    except (OSError, ValueError) as e:
        return {"status": f"no trained weights ({e})"}
    stream = torch.cuda.current_stream()
    net = P.FNet(params)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    plain_s = learned_s = 0.0
    reached, ratios, fb_ratios = 0, [], []
    qcap = 15
    plan = P.Plan(1024, 1024, LR._dummy_psf(qcap), dtype="f32")
    plan.ar_plan_autotune()
    for i in range(images):
        F, H, E, prm = synth.learned_problem(i, n=1024, base_seed=6_000_000)
        plan.ar_plan_set_psf(H)
        f, g = LR.observe_gpu(plan, F, E, prm["nu"], torch.float32)
        x = torch.zeros_like(g)
        torch.cuda.synchronize()
        best = np.inf
        ev[0].record(stream)
        for kind, prm_s in LR.SETTINGS:
            plan.ar_precond_set(kind, prm_s)
            x.zero_()
            _, _, rre, _ = plan.ar_deblur_iterate(g, x, iters, f_true=f, want_rre=True)
            m = finite_min(rre)
            if m is not None:
                best = min(best, m)
        ev[1].record(stream)
        torch.cuda.synchronize()
        plain_s += ev[0].elapsed_time(ev[1]) / 1e3
        x.zero_()
        torch.cuda.synchronize()
        ev[0].record(stream)
        LR.apply_learned(net, plan, g)
        ev[1].record(stream)
        _, _, rre, _ = plan.ar_deblur_iterate(g, x, iters, f_true=f, want_rre=True)
        ev[2].record(stream)
        torch.cuda.synchronize()
        t_setup = ev[0].elapsed_time(ev[1]) / 1e3
        t_run = ev[1].elapsed_time(ev[2]) / 1e3
        ok = np.nonzero(np.isfinite(rre) & (rre <= 1.02 * best))[0]
        if ok.size:
            reached += 1
            learned_s += t_setup + t_run * (ok[0] + 1) / iters
        else:
            learned_s += t_setup + t_run
        mb = finite_min(rre)
        ratios.append((mb if mb is not None else np.inf) / best)
        plan.ar_precond_set(*LR.FALLBACK)
        x.zero_()
        _, _, rre, _ = plan.ar_deblur_iterate(g, x, iters, f_true=f, want_rre=True)
        mb = finite_min(rre)
        fb_ratios.append((mb if mb is not None else np.inf) / best)
    plan.close()
    net.close()
    return {"images": images, "n": 1024, "iterations": iters,
            "plain_sweep_gpu_s": round(plain_s, 4), "learned_gpu_s": round(learned_s, 4),
            "speedup": round(plain_s / learned_s, 2) if learned_s > 0 else None,
            "reached_within_2pct": reached,
            "median_best_rre_ratio_learned": round(float(np.median(ratios)), 4),
            "median_best_rre_ratio_fallback": round(float(np.median(fb_ratios)), 4),
            "workload": "1024x1024 phantoms, PSFs 15..31 (motion / exponential tail / "
                        "shifted Gaussian), noise log-uniform 0.1%..2%, seeds 6,000,000 + i"}


def bench_precision(torch, P, iters):
    """The precision variant: 2048^2 FP32 images, 31x31 one-sided
    exponential-tail PSF, 1% noise, Tikhonov alpha 5e-3, `iters` iterations
    with every transform pass as a BF16x3 MFMA GEMM (AR_F32_BF16X3).  Its
    error is reported against the FP64-arithmetic GPU path (AR_F64 on the
    same data; that path matches the FP64 oracle to 1e-12): relative
    difference of x_1 and x_10, and the best RRE of both runs."""
    import synth
    F, H, E, p = synth.workload("ar2048_f32_tail31")
    n = p["n"]
    plan = P.Plan(n, n, H, dtype="bf16x3")
    plan.ar_precond_set(P.AR_FILTER_TIKHONOV, p["alpha"])
    f = torch.from_numpy(F).to("cuda:0", torch.float32)
    e = torch.from_numpy(E).to("cuda:0", torch.float32)
    b = torch.empty_like(f)
    plan.ar_blur_apply(f, b)
    g = b + (p["nu"] * torch.linalg.vector_norm(b.double()) /
             torch.linalg.vector_norm(e.double())).float() * e
    x = torch.zeros_like(g)
    plan.ar_deblur_iterate(g, x, 5)                  # warm-up
    x.zero_()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    rc, res, _, _ = plan.ar_deblur_iterate(g, x, iters, want_resnorm=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    t = ev0.elapsed_time(ev1) / 1e3
    out = {"workload": "2048x2048 phantom (40 blobs + 20 rectangles, seed 303), 31x31 one-sided "
                       "exponential tail exp(-s1/4) x Gaussian sigma 2, 1% noise, Tikhonov alpha "
                       "5e-3, BF16x3 MFMA transforms, FP32 blur, FP64 eigenvalues/filter/norms",
           "iterations": iters, "value": round(n * n * iters / t / 1e6, 1),
           "unit": "Mpixel-iters/s", "ms_per_iteration": round(t / iters * 1e3, 4),
           "status": rc}
    ref = P.Plan(n, n, H, dtype="f64")
    ref.ar_precond_set(P.AR_FILTER_TIKHONOV, p["alpha"])
    g64, f64 = g.double(), f.double()
    errs = {}
    xb = torch.zeros_like(g)
    xr = torch.zeros_like(g64)
    done = 0
    for k in (1, 10):
        plan.ar_deblur_iterate(g, xb, k - done)
        ref.ar_deblur_iterate(g64, xr, k - done)
        done = k
        errs[f"x{k}_rel_err_vs_f64"] = float(torch.linalg.vector_norm(xb.double() - xr) /
                                            torch.linalg.vector_norm(xr))
    xb.zero_()
    xr.zero_()
    _, _, rre_b, best_b = plan.ar_deblur_iterate(g, xb, iters, f_true=f, want_rre=True)
    _, _, rre_r, best_r = ref.ar_deblur_iterate(g64, xr, iters, f_true=f64, want_rre=True)
    out.update(errs)
    out.update({"best_rre": finite_min(rre_b), "best_it": best_b,
                "f64_best_rre": finite_min(rre_r), "f64_best_it": best_r})
    # per operator, on the phantom: T~ f, T (T~ f) and the preconditioner
    # solve, each against the FP64 plan on the same FP32 input
    ops = {}
    cb, cr = torch.empty_like(f), torch.empty_like(f64)
    plan.ar_transform(f, cb)
    ref.ar_transform(f64, cr)
    ops["transform_rel_err_vs_f64"] = float(torch.linalg.vector_norm(cb.double() - cr) /
                                            torch.linalg.vector_norm(cr))
    yb, yr = torch.empty_like(f), torch.empty_like(f64)
    plan.ar_transform_inv(cb, yb)
    ref.ar_transform_inv(cb.double(), yr)
    ops["transform_inv_rel_err_vs_f64"] = float(torch.linalg.vector_norm(yb.double() - yr) /
                                                torch.linalg.vector_norm(yr))
    plan.ar_precond_solve(f, yb)
    ref.ar_precond_solve(f64, yr)
    ops["precond_solve_rel_err_vs_f64"] = float(torch.linalg.vector_norm(yb.double() - yr) /
                                                torch.linalg.vector_norm(yr))
    out["per_operator"] = ops
    plan.close()
    ref.close()
    return out


def bench_bc_variants(torch, P, F, H, E, p, iters=ITERS, steps=500, reps=100):
    """The comparators of the paper's tables on the same 1024^2 workload at
    the stable alpha: D-Landweber under Reflective BCs (DCT-III algebra)
    and under Periodic BCs (FFT), FP32; and the direct Tikhonov solve of
    the strongly symmetric (4-fold symmetrized) PSF under Anti-Reflective
    and Reflective BCs.  Each iteration's per-phase kernel times and the
    step-level HBM fraction use the same algorithmic bytes as the timed
    Anti-Reflective run (36 B per pixel-iteration)."""
    import oracle as O
    n = p["n"]
    out = {}
    f = torch.from_numpy(F).to("cuda:0", torch.float32)
    e = torch.from_numpy(E).to("cuda:0", torch.float32)
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    for bc in ("reflective", "periodic"):
        plan = P.Plan(n, n, H, dtype="f32", bc=bc)
        b = torch.empty_like(f)
        plan.ar_blur_apply(f, b)
        g = b + (p["nu"] * torch.linalg.vector_norm(b.double()) /
                 torch.linalg.vector_norm(e.double())).float() * e
        plan.ar_precond_set(P.AR_FILTER_TIKHONOV, STABLE_ALPHA)
        x = torch.zeros_like(g)
        plan.ar_deblur_iterate(g, x, iters, want_resnorm=True)          # warm-up
        torch.cuda.synchronize()
        ev0.record(stream)
        done, rc = 0, 0
        while done < steps:
            k = min(iters, steps - done)
            x.zero_()
            rck, _, _, _ = plan.ar_deblur_iterate(g, x, k, want_resnorm=True)
            rc = rc or rck
            done += k
        ev1.record(stream)
        torch.cuda.synchronize()
        t = ev0.elapsed_time(ev1) / 1e3 / steps
        x.zero_()
        rcq, res, rre, best = plan.ar_deblur_iterate(g, x, iters, f_true=f, want_resnorm=True,
                                                     want_rre=True)
        ph = plan.ar_iterate_profile(g, x, reps=reps)
        gbs = STEP_BYTES * n * n / t / 1e9
        out[bc] = {"value": round(n * n / t / 1e6, 1), "unit": "Mpixel-iters/s",
                   "us_per_step": round(t * 1e6, 2), "status": rc,
                   "best_it": best, "best_rre": finite_min(rre), "diverged": diverged(res),
                   "phase_us": [round(v, 2) for v in ph],
                   "step_roofline": {"bound": "hbm", "achieved": round(gbs, 2),
                                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": round(gbs / HBM_PEAK_GBS, 4)}}
        plan.close()
    S = O.symmetrize(H)
    for bc in ("antireflective", "reflective"):
        plan = P.Plan(n, n, S, dtype="f32", bc=bc)
        b = torch.empty_like(f)
        plan.ar_blur_apply(f, b)
        xs = torch.empty_like(b)
        plan.ar_tikhonov_solve(b, xs, 5e-3)                               # warm-up
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(reps):
            plan.ar_tikhonov_solve(b, xs, 5e-3)
        ev1.record(stream)
        torch.cuda.synchronize()
        t = ev0.elapsed_time(ev1) / 1e3 / reps
        # algorithmic bytes of one solve: read g, write x (FP32), read lambda (FP64)
        gbs = (4 + 4 + 8) * n * n / t / 1e9
        out[f"tikhonov_solve_{bc}"] = {
            "us_per_solve": round(t * 1e6, 2), "value": round(n * n / t / 1e6, 1),
            "unit": "Mpixel/s", "rre": float(torch.linalg.vector_norm(xs.double() - f.double()) /
                                             torch.linalg.vector_norm(f.double())),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "bytes_per_pixel": 16}}
        plan.close()
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); "
              "the multi-GPU sharding is a design, not part of this build", file=sys.stderr)
        return 2
    import torch
    import paper_1211_0393_amd as P
    P.load()                                            # fail loudly without the HIP library
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    plan, f, g, F, H, E, p = make_inputs(torch, P, a.dtype)
    plan.ar_precond_set(P.AR_FILTER_TIKHONOV, a.alpha)
    n = p["n"]
    stream = torch.cuda.current_stream()
    keys = {"row_waves": P.AR_TUNE_ROW_WAVES, "col_waves": P.AR_TUNE_COL_WAVES,
            "row_excl": P.AR_TUNE_ROW_EXCL, "col_excl": P.AR_TUNE_COL_EXCL,
            "row_fft": P.AR_TUNE_ROW_ALGO, "col_fft": P.AR_TUNE_COL_ALGO,
            "row_lanes": P.AR_TUNE_ROW_LANES, "col_lanes": P.AR_TUNE_COL_LANES,
            "blur_engine": P.AR_TUNE_BLUR}
    tuned_us = None
    if a.tuning:
        for k, v in json.loads(a.tuning).items():
            if k in keys:
                plan.ar_plan_tune(keys[k], int(v))
    elif not a.no_tune:
        tuned_us = plan.ar_plan_autotune()
    tuning = {k: plan.ar_plan_get_tune(v) for k, v in keys.items()}
    x = torch.zeros_like(g)

    def runs(total):
        # the workload is a run of ITERS iterations from x = 0; `total` steps
        # are that many consecutive runs (the last one possibly shorter)
        return [min(ITERS, total - k) for k in range(0, total, ITERS)]

    # warm-up (untimed), in the same run lengths as the timed loop
    for k in runs(max(a.warmup, min(a.steps, ITERS))):
        x.zero_()
        plan.ar_deblur_iterate(g, x, k, want_resnorm=True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    rc, res = 0, None
    for k in runs(a.steps):
        x.zero_()
        rck, res, _, _ = plan.ar_deblur_iterate(g, x, k, want_resnorm=True)
        rc = rc or rck
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    t_step = max(wall, gpu_s) / a.steps
    value = n * n / t_step / 1e6

    # quality of the timed run, of the named alpha's run and of the
    # unpreconditioned reference run, each ITERS iterations
    x.zero_()
    rc_t, res_t, rre_t, best_t = plan.ar_deblur_iterate(g, x, ITERS, f_true=f,
                                                        want_resnorm=True, want_rre=True)
    plan.ar_precond_set(P.AR_FILTER_TIKHONOV, p["alpha"])
    x.zero_()
    rc_q, res_q, rre, best = plan.ar_deblur_iterate(g, x, ITERS, f_true=f, want_resnorm=True,
                                                    want_rre=True)
    plan.ar_precond_set(P.AR_FILTER_TIKHONOV, a.alpha)
    xr = torch.zeros_like(g)
    rc_p, res_p, rre_p, best_p = plan.ar_deblur_iterate(g, xr, ITERS, precondition=False,
                                                        f_true=f, want_resnorm=True,
                                                        want_rre=True)

    # per-kernel durations of one step (HIP events on this stream, around
    # back-to-back launches of each phase kernel), and the rooflines with the
    # algorithmic work per launch: the blur kernels are bound by the vector
    # ALU (2 P flops per pixel in the plan's arithmetic type), the transform
    # passes by HBM with the algorithmic bytes they own
    phase_us = plan.ar_iterate_profile(g, x, reps=a.kernel_reps)
    blur_engines = None
    if a.dtype == "f32":
        # both FP32 blur engines timed on the same plan and data
        keep = plan.ar_plan_get_tune(P.AR_TUNE_BLUR)
        blur_engines = {}
        for name, eng in (("vector_alu", 1), ("matrix_cores", 2)):
            try:
                plan.ar_plan_tune(P.AR_TUNE_BLUR, eng)
            except P.ArError:
                continue
            us = plan.ar_iterate_profile(g, x, reps=a.kernel_reps)
            blur_engines[name] = {"residual_us": round(us[0], 2), "reblur_us": round(us[1], 2)}
        plan.ar_plan_tune(P.AR_TUNE_BLUR, keep)
    P_taps = (2 * plan.q1 + 1) * (2 * plan.q2 + 1)
    npx = n * n
    alu_peak = FP64_VECTOR_TFLOPS if a.dtype == "f32x" else FP32_VECTOR_TFLOPS
    alu_kind = "FP64 vector" if a.dtype == "f32x" else "FP32 vector"
    phases = [
        ("residual blur r = g - A x", "alu", 2.0 * P_taps * npx, ALG_BYTES["residual"] * npx),
        ("reblur y = A' r", "alu", 2.0 * P_taps * npx, ALG_BYTES["reblur"] * npx),
        ("row pass of T~", "hbm", None, ALG_BYTES["row_fwd"] * npx),
        ("column pass T~, d, T", "hbm", None, ALG_BYTES["col"] * npx),
        ("row pass of T + update", "hbm", None, ALG_BYTES["row_inv"] * npx),
    ]
    traffic = measured_traffic(a.dtype)
    rooflines = []
    for (name, bound, flops, nbytes), us in zip(phases, phase_us):
        t = us * 1e-6
        if bound == "alu":
            ach, peak, unit = flops / t / 1e12, alu_peak, "TFLOP/s"
        else:
            ach, peak, unit = nbytes / t / 1e9, HBM_PEAK_GBS, "GB/s"
        rooflines.append({"kernel": name, "bound": bound, "achieved": round(ach, 2), "peak": peak,
                          "unit": unit, "frac": round(ach / peak, 4),
                          "traffic": traffic.get(name),
                          "kernel_us": round(us, 2),
                          "algorithmic": {"flops": flops, "bytes": nbytes},
                          **({"peak_kind": alu_kind} if bound == "alu" else {})})
    dom = int(np.argmax(phase_us))
    roof = dict(rooflines[dom])
    step_gbs = STEP_BYTES * npx / t_step / 1e9
    step_roof = {"bound": "hbm", "achieved": round(step_gbs, 2), "peak": HBM_PEAK_GBS,
                 "unit": "GB/s", "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                 "bytes_per_pixel_iteration": STEP_BYTES, "us_per_step": round(t_step * 1e6, 2)}
    fpx = step_flops(n, n, P_taps)
    step_tf = fpx * npx / t_step / 1e12
    step_alu = {"bound": "alu", "achieved": round(step_tf, 2), "peak": alu_peak,
                "unit": "TFLOP/s", "frac": round(step_tf / alu_peak, 4), "peak_kind": alu_kind,
                "flops_per_pixel_iteration": round(fpx, 1)}

    net_path = None
    if a.learned_images >= 0:
        from paper_1211_0393_amd import learned as LR
        net_path = LR.WEIGHTS if os.path.exists(LR.WEIGHTS) else None
    stable = bench_stable(torch, P, plan, f, g, net_path)
    plan.ar_precond_set(P.AR_FILTER_TIKHONOV, a.alpha)
    bc_variants = None if a.no_bc else bench_bc_variants(torch, P, F, H, E, p)
    batch = None if a.no_batch else bench_batch(torch, P, ITERS)
    learned = bench_learned(torch, P, a.learned_images, ITERS) if a.learned_images > 0 else None
    precision = None if a.no_precision else bench_precision(torch, P, 200)
    if a.copy_probe:
        src = torch.ones(64 << 20, device="cuda:0", dtype=torch.float32)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    cpu = None
    if not a.no_cpu and int(os.environ.get("RANK", "0")) == 0:
        cpu = cpu_baseline(F, H, E, p, a.cpu_iters)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpixel-iters/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(t_step * 1e3, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32 images, f64 arithmetic (the inverse row pass after the filter in f32)"
                  if a.dtype == "f32x" else "f32"),
        "data": "synthetic",
        "config": {"workload": "1024x1024 phantom (40 blobs + 20 rectangles), 15x15 motion PSF "
                               "(length 11 at 30 deg, Gaussian sigma 1), 0.5% noise, AR BCs, "
                               f"D-Landweber with Tikhonov alpha {a.alpha} (the named 5e-3 "
                               "diverges, see quality), reblur transpose, tau 1",
                   "n1": n, "n2": n, "psf": [15, 15], "alpha": a.alpha,
                   "named_alpha": p["alpha"], "iterations": ITERS, "parallelism": "single GPU"},
        "status": rc,
        "timed_run": {"alpha": a.alpha, "status": rc_t, "best_it": best_t,
                      "best_rre": finite_min(rre_t), "diverged": diverged(res_t) or diverged(res)},
        "quality": {"alpha": p["alpha"], "status": rc_q, "best_it": best,
                    "best_rre": finite_min(rre), "diverged": diverged(res_q),
                    "plain_best_it": best_p, "plain_best_rre": finite_min(rre_p),
                    "plain_diverged": diverged(res_p),
                    "note": "at alpha 5e-3 D-Landweber is unstable for this PSF (I - D A'A has "
                            "spectral radius ~7); throughput does not depend on alpha; "
                            "stable_alpha holds the restoration comparison"},
        "stable_alpha": stable,
        "tuning": dict(tuning, iteration_us=tuned_us),
        "roofline": roof,
        "step_roofline": step_roof,
        "step_alu_roofline": step_alu,
        "kernels": rooflines,
        "blur_engines": blur_engines,
        "cpu_baseline": cpu,
        "boundary_conditions": bc_variants,
        "batch": batch,
        "learned_vs_plain": learned,
        "precision_variant": precision,
    }
    print(json.dumps(out, allow_nan=False), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
