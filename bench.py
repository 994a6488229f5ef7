#!/usr/bin/env python3
"""Benchmark: D-Landweber under AR boundary conditions on one MI355X.

A step is one pass of the whole hot path over the 1024x1024 workload:
residual r = g - A x (AR blur, FP64 norm partials), y = A' r (reblur),
c = T~ y along rows, the fused column pass T~ / filter d / T, and the row
pass T fused with x += tau w, i.e. one preconditioned Landweber iteration
including its per-iteration FP64 residual norm.  The timed region runs
exactly K steps from x_0 = 0 with all inputs resident on the GPU; the
per-iteration norms are copied to the host once at the end (inside the
timed region).

Prints one JSON line (see the repository's design notes for the roofline
and the CPU baseline definitions).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f32x|f32]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "Mpixel-iters/s at 1024² FP32 + GPU time to best rel. error, learned vs plain"
WORKLOAD = "ar1024_f32_motion15"
ITERS = 100   # iterations of one run of the workload (its configuration)

# MI355X published peaks used for the roofline (dense, per GPU)
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = 78.6   # FP64 vector, and FP32 vector without packed FP32
                          # (256 CUs x 64 FMA lanes/clk x 2 flop x 2.4 GHz)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000,
                    help="timed iterations, run as consecutive runs of at most 100 from x = 0")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--dtype", default="f32x", choices=["f32x", "f32"])
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--no-tune", action="store_true", help="skip the plan autotuner")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
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
    plan.ar_precond_set(P.AR_FILTER_TIKHONOV, p["alpha"])
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


def finite_min(v):
    if v is None:
        return None
    v = np.asarray(v)
    v = v[np.isfinite(v)]
    return float(v.min()) if v.size else None


def cpu_baseline(F, H, E, p, iters):
    """The FP64 oracle (as written, untuned) on this host: a bounded sample
    of the same workload (`iters` D-Landweber iterations after one warm-up
    iteration), in Mpixel-iters/s."""
    import oracle as O
    G = O.observe(F, H, E, p["nu"])
    d = O.tikhonov(O.eigenvalues(H, *G.shape), p["alpha"])
    X = np.zeros_like(G)
    X, _ = O.landweber_step(X, G, H, d=d)          # warm-up
    t0 = time.perf_counter()
    for _ in range(iters):
        X, _ = O.landweber_step(X, G, H, d=d)
    dt = time.perf_counter() - t0
    px = G.size * iters
    return {"value": px / dt / 1e6, "unit": "Mpixel-iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} FP64 D-Landweber iterations of the 1024x1024 15x15-PSF workload "
                      f"after 1 warm-up ({dt:.1f} s); numpy/scipy single-threaded "
                      f"(host os.cpu_count()={os.cpu_count()})"}


def bench_batch(torch, P, iters, count=256):
    """The batched workload: `count` problems (n in {128,...,512}, own
    Gaussian PSF 7..21 and noise level, Tikhonov alpha 5e-3, FP32), `iters`
    preconditioned iterations in one graph launch, after a warm-up call
    that captures the graph.  Inputs are resident on the GPU."""
    import synth
    plans, gs, xs = [], [], []
    px = 0
    for i in range(count):
        F, H, E, prm = synth.batch_problem(i)
        n = prm["n"]
        pl = P.Plan(n, n, H, dtype="f32")
        pl.ar_precond_set(P.AR_FILTER_TIKHONOV, prm["alpha"])
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
    batch.ar_batch_iterate(gs, xs, iters)            # warm-up: captures the graph
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
    out = {"workload": f"{count} problems, n in {{128,192,256,384,512}} (seed 404 + i), "
                       "Gaussian PSFs 7..21, noise 0.1%..2%, Tikhonov alpha 5e-3, FP32, "
                       f"{iters} D-Landweber iterations in one graph launch",
           "value": round(px * iters / t / 1e6, 1), "unit": "Mpixel-iters/s",
           "pixels_per_iteration": px, "seconds": round(t, 5),
           "us_per_batch_iteration": round(t / iters * 1e6, 2),
           "status": rc, "autotuned_precond_us": round(tuned, 2),
           "diverged_problems": int(np.sum(~np.all(np.isfinite(res), axis=1)))}
    batch.close()
    for pl in plans:
        pl.close()
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
    plan.close()
    ref.close()
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
    n = p["n"]
    stream = torch.cuda.current_stream()
    tuned_us = plan.ar_plan_autotune() if not a.no_tune else None
    tuning = {k: plan.ar_plan_get_tune(v) for k, v in
              [("row_waves", P.AR_TUNE_ROW_WAVES), ("col_waves", P.AR_TUNE_COL_WAVES),
               ("row_excl", P.AR_TUNE_ROW_EXCL), ("col_excl", P.AR_TUNE_COL_EXCL),
               ("row_fft", P.AR_TUNE_ROW_ALGO), ("col_fft", P.AR_TUNE_COL_ALGO),
               ("row_lanes", P.AR_TUNE_ROW_LANES), ("col_lanes", P.AR_TUNE_COL_LANES)]}
    x = torch.zeros_like(g)

    def runs(total):
        # the workload is a run of ITERS iterations from x = 0; `total` steps
        # are that many consecutive runs (the last one possibly shorter)
        return [min(ITERS, total - k) for k in range(0, total, ITERS)]

    # warm-up (untimed)
    for k in runs(a.warmup):
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

    # quality of the timed run and of the unpreconditioned reference run
    x.zero_()
    rc_q, _, rre, best = plan.ar_deblur_iterate(g, x, ITERS, f_true=f, want_rre=True)
    xr = torch.zeros_like(g)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rc_p, _, rre_p, best_p = plan.ar_deblur_iterate(g, xr, ITERS, precondition=False,
                                                    f_true=f, want_rre=True)
    plain_s = time.perf_counter() - t1

    # per-kernel durations of one step (HIP events on this stream), and the
    # roofline of the dominant kernel with its algorithmic work per launch
    phase_us = plan.ar_iterate_profile(g, x, reps=a.kernel_reps)
    P_taps = (2 * plan.q1 + 1) * (2 * plan.q2 + 1)
    npx = n * n
    es = 4                                           # FP32 images
    ds = es                                          # filter (transposed) in the storage type
    phases = [
        ("residual blur r = g - A x", "alu", 2.0 * P_taps * npx, 3 * es * npx, "conv_kernel"),
        ("reblur y = A' r", "alu", 2.0 * P_taps * npx, 2 * es * npx, "conv_kernel"),
        ("row pass of T~", "hbm", None, 2 * es * npx, "rows_w_kernel"),
        ("column pass T~, d, T", "hbm", None, (2 * es + ds) * npx, "cols_w_kernel"),
        ("row pass of T + update", "hbm", None, 3 * es * npx, "rows_w_kernel"),
    ]
    traffic = measured_traffic(a.dtype)
    rooflines = []
    for (name, bound, flops, nbytes, kname), us in zip(phases, phase_us):
        t = us * 1e-6
        if bound == "alu":
            ach, peak, unit = flops / t / 1e12, VALU_PEAK_TFLOPS, "TFLOP/s"
        else:
            ach, peak, unit = nbytes / t / 1e9, HBM_PEAK_GBS, "GB/s"
        rooflines.append({"kernel": name, "bound": bound, "achieved": round(ach, 2), "peak": peak,
                          "unit": unit, "frac": round(ach / peak, 4),
                          "traffic": traffic.get(name),
                          "kernel_us": round(us, 2),
                          "algorithmic": {"flops": flops, "bytes": nbytes}})
    dom = int(np.argmax(phase_us))
    roof = dict(rooflines[dom])
    roof["hbm_frac_of_step"] = round(npx * 36 / t_step / 1e9 / HBM_PEAK_GBS, 4)

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
                               "D-Landweber with Tikhonov alpha 5e-3, reblur transpose, tau 1",
                   "n1": n, "n2": n, "psf": [15, 15], "alpha": p["alpha"],
                   "iterations": ITERS, "parallelism": "single GPU"},
        "status": rc,
        "quality": {"best_it": best, "best_rre": finite_min(rre),
                    "plain_best_it": best_p, "plain_best_rre": finite_min(rre_p),
                    "plain_run_s": round(plain_s, 5),
                    "diverged": bool(res is not None and not np.all(np.isfinite(res)))},
        "tuning": dict(tuning, iteration_us=tuned_us),
        "roofline": roof,
        "kernels": rooflines,
        "cpu_baseline": cpu,
        "batch": batch,
        "learned_vs_plain": learned,
        "precision_variant": precision,
    }
    print(json.dumps(out, allow_nan=False), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
