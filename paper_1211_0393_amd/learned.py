"""Learned preconditioner filter: label sweeps, training and inference.

Every numerical step runs in the HIP library: the plain-method sweeps run
through the batched executor (ar_batch_iterate), features, gains, labels
and the network's forward, backward and Adam steps through ar_features,
ar_precond_set_gains, ar_gains_label and ar_fnet_*.  This module only
orders the calls, moves tensors and keeps the bookkeeping.

Label of a problem: among 16 Tikhonov parameters (log-spaced in
[1e-3, 1]) and 16 threshold parameters (log-spaced in [1e-2, 0.9]) the
plain filter whose D-Landweber run reaches the smallest relative
restoration error within K iterations; its label (ar_gains_label) is the
per-eigenvalue-bin Tikhonov parameter that reproduces that filter.  The
fallback filter is Tikhonov at the sweep's 13th parameter (about 0.25), the
Tikhonov parameter most often best on the 256^2 and 1024^2 training labels.

The committed weights (fnet_weights.npy) come from

    python -m paper_1211_0393_amd.learned --tuples 8000 --n 256 --steps 0 \
        --save-data learned_256.npz
    python -m paper_1211_0393_amd.learned --tuples 2800 --n 1024 --chunk 4 \
        --steps 0 --save-data learned_1024.npz
    python -m paper_1211_0393_amd.learned --data learned_256.npz learned_1024.npz \
        --limit 0 2400 --repeat 1 3 --steps 8000 --seed 3

(training problems 5,000,000 + i; the last 400 problems at 1024^2 were kept
out of training for validation).
"""

from __future__ import annotations

import argparse
import time

import numpy as np

from . import _lib as L

ALPHAS = np.logspace(-3, 0, 16)
THRESHOLDS = np.logspace(-2, np.log10(0.9), 16)
SETTINGS = [(L.AR_FILTER_TIKHONOV, float(a)) for a in ALPHAS] + \
           [(L.AR_FILTER_THRESHOLD, float(t)) for t in THRESHOLDS]
FALLBACK = (L.AR_FILTER_TIKHONOV, float(ALPHAS[12]))
WEIGHTS = __file__.rsplit("/", 1)[0] + "/fnet_weights.npy"


def _torch():
    import torch
    return torch


def observe_gpu(plan, F, E, nu, dtype):
    """g = A f + nu ||A f|| e / ||e|| with the blur on the GPU."""
    torch = _torch()
    f = torch.from_numpy(np.ascontiguousarray(F)).to("cuda:0", dtype)
    e = torch.from_numpy(np.ascontiguousarray(E)).to("cuda:0", dtype)
    b = torch.empty_like(f)
    plan.ar_blur_apply(f, b)
    scale = (nu * torch.linalg.vector_norm(b.double()) / torch.linalg.vector_norm(e.double()))
    return f, b + scale.to(dtype) * e


def _dummy_psf(q):
    H = np.zeros((2 * q + 1, 2 * q + 1))
    H[q, q] = 1.0
    return H


def sweep_labels(problems, K=100, chunk=8, dtype="f32", log=None, qcap=None):
    """Features (N x 65), labels (N x 64), best RRE and best setting index of
    each problem (F, H, E, nu) by the plain sweep; all problems share one
    size n x n.  ``problems`` is a sequence (or an object with __len__ and
    __getitem__ that builds problems on demand); ``qcap`` bounds the PSF
    half-widths (default: the largest of the sequence)."""
    torch = _torch()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    n = problems[0][0].shape[0]
    S = len(SETTINGS)
    if qcap is None:
        qcap = max(max(H.shape) for (_, H, _, _) in problems) // 2
    pool = [L.Plan(n, n, _dummy_psf(qcap), dtype=dtype) for _ in range(chunk * S)]
    N = len(problems)
    feats = torch.zeros((N, L.AR_FNET_IN), device="cuda:0", dtype=torch.float32)
    labels = torch.zeros((N, L.AR_FNET_BINS), device="cuda:0", dtype=torch.float32)
    best_rre = np.full(N, np.inf)
    best_set = np.zeros(N, dtype=np.int64)
    t0 = time.perf_counter()
    try:
        for c0 in range(0, N, chunk):
            sub = [problems[i] for i in range(c0, min(N, c0 + chunk))]
            plans = pool[:len(sub) * S]
            gs, fs = [], []
            for j, (F, H, E, nu) in enumerate(sub):
                for s, (kind, prm) in enumerate(SETTINGS):
                    pl = plans[j * S + s]
                    pl.ar_plan_set_psf(H)
                    pl.ar_precond_set(kind, prm)
                f, g = observe_gpu(plans[j * S], F, E, nu, tdt)
                plans[j * S].ar_features(g, feats[c0 + j])
                gs += [g] * S
                fs += [f] * S
            xs = [torch.zeros_like(g) for g in gs]
            with L.Batch(plans) as b:
                _, _, rre, _ = b.ar_batch_iterate(gs, xs, K, f_true=fs, want_rre=True)
            rre = np.where(np.isfinite(rre), rre, np.inf).min(axis=1)
            for j in range(len(sub)):
                r = rre[j * S:(j + 1) * S]
                s = int(np.argmin(r))
                best_rre[c0 + j] = r[s]
                best_set[c0 + j] = s
                plans[j * S + s].ar_gains_label(labels[c0 + j])
            if log and (c0 // chunk) % 20 == 0:
                log(f"labels {c0 + len(sub)}/{N} ({time.perf_counter() - t0:.1f} s)")
    finally:
        for pl in pool:
            pl.close()
    torch.cuda.synchronize()
    return feats, labels, best_rre, best_set


def init_params(seed=0):
    """He-normal weights, zero biases (FP32), in the network's layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for (o, i) in [(L.AR_FNET_HIDDEN, L.AR_FNET_IN), (L.AR_FNET_HIDDEN, L.AR_FNET_HIDDEN),
                   (L.AR_FNET_BINS, L.AR_FNET_HIDDEN)]:
        parts.append(rng.standard_normal(o * i) * np.sqrt(2.0 / i))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def train(feats, labels, steps=2000, batch=256, lr=1e-3, seed=0, log=None):
    """Adam training of a fresh network on device tensors (N x 65, N x 64);
    returns the network."""
    torch = _torch()
    net = L.FNet(init_params(seed))
    N = feats.shape[0]
    rng = np.random.default_rng(seed + 1)
    loss = torch.zeros(1, device="cuda:0", dtype=torch.float32)
    order = rng.permutation(N)
    pos = 0
    for it in range(steps):
        if pos + min(batch, N) > N:
            order = rng.permutation(N)
            pos = 0
        idx = torch.from_numpy(order[pos:pos + min(batch, N)]).to("cuda:0")
        pos += min(batch, N)
        net.ar_fnet_train_step(feats[idx].contiguous(), labels[idx].contiguous(), lr, loss)
        if log and (it % 500 == 0 or it == steps - 1):
            torch.cuda.synchronize()
            log(f"step {it}: loss {loss.item():.5f}")
    torch.cuda.synchronize()
    return net


def apply_learned(net, plan, g):
    """Features of (plan, g) -> network -> gains filter of the plan."""
    torch = _torch()
    feat = torch.empty((1, L.AR_FNET_IN), device="cuda:0", dtype=torch.float32)
    plan.ar_features(g, feat)
    gains = torch.empty((1, L.AR_FNET_BINS), device="cuda:0", dtype=torch.float32)
    net.ar_fnet_infer(feat, gains)
    plan.ar_precond_set_gains(gains)
    return gains


def save_params(path, params):
    np.save(path, np.asarray(params, dtype=np.float32), allow_pickle=False)


def load_params(path=WEIGHTS):
    p = np.load(path, allow_pickle=False)
    if p.shape != (L.AR_FNET_NPARAM,) or p.dtype != np.float32:
        raise ValueError(f"{path}: not a filter-network parameter vector")
    return p


class Problems:
    """Training problems built on demand (synth.learned_problem)."""

    def __init__(self, count, n=256, seed0=5_000_000, sizes=None, first=0):
        self.count, self.n, self.seed0, self.sizes, self.first = count, n, seed0, sizes, first

    def __len__(self):
        return self.count

    def __getitem__(self, i):
        import synth
        kw = {} if self.sizes is None else {"sizes": self.sizes}
        F, H, E, prm = synth.learned_problem(self.first + i, n=self.n, base_seed=self.seed0, **kw)
        return F, H, E, prm["nu"]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--tuples", type=int, default=20000)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--chunk", type=int, default=8)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed0", type=int, default=5_000_000)
    ap.add_argument("--first", type=int, default=0, help="index of the first problem")
    ap.add_argument("--data", nargs="*", default=[],
                    help="train on saved features/labels (.npz) instead of sweeping")
    ap.add_argument("--limit", nargs="*", type=int, default=[],
                    help="per --data file: use its first N examples (0 = all)")
    ap.add_argument("--repeat", nargs="*", type=int, default=[],
                    help="per --data file: how many times its examples enter the set")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--save-data", default=None, help="also save features/labels (.npz)")
    a = ap.parse_args(argv)
    L.load()

    def log(m):
        print(m, flush=True)

    torch = _torch()
    if a.data:
        fs, ls = [], []
        for k, f in enumerate(a.data):
            part = np.load(f, allow_pickle=False)
            lim = a.limit[k] if k < len(a.limit) and a.limit[k] > 0 else None
            rep = a.repeat[k] if k < len(a.repeat) else 1
            fs += [part["feats"][:lim]] * rep
            ls += [part["labels"][:lim]] * rep
        feats = torch.from_numpy(np.concatenate(fs)).to("cuda:0")
        labels = torch.from_numpy(np.concatenate(ls)).to("cuda:0")
        log(f"{feats.shape[0]} saved examples loaded")
    else:
        probs = Problems(a.tuples, a.n, a.seed0, first=a.first)
        feats, labels, best, sel = sweep_labels(probs, K=a.iters, chunk=a.chunk, log=log, qcap=15)
        log(f"labels done; mean best RRE {np.mean(best):.4f}; "
            f"Tikhonov chosen {np.mean(sel < 16):.2f} of the time")
        if a.save_data:
            np.savez(a.save_data, feats=feats.cpu().numpy(), labels=labels.cpu().numpy(),
                     best=best, sel=sel)
    if a.steps <= 0:
        return
    net = train(feats, labels, steps=a.steps, batch=a.batch, lr=a.lr, seed=a.seed, log=log)
    save_params(a.out, net.ar_fnet_get_params())
    log(f"saved {a.out}")


if __name__ == "__main__":
    main()
