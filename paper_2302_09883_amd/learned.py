"""Learned per-patch thresholds on the D2Q9 workload (GPU).

The paper sets one threshold constant per run by hand for an error target
(Section 2.2, Section 3.2).  Here a small network chooses one per patch:

* **Data** from the plain method's own runs: a compressed D2Q9 run (double
  shear layer plus seeded vortices) is stopped at several times; from each
  stopped state, every candidate threshold is run for a window of T steps
  next to the uncompressed scheme started from the same decompressed state.
  Per patch: the network input of the stopped state (its stored
  coefficients at stride 8, ``Context.features``), and per candidate the
  squared error the window added and the bytes of the patch's records.
* **Network** (``Net``, hand-written HIP kernels, bfloat16 weights): input ->
  2 K outputs, the log10 squared error and log10 record bytes per candidate;
  trained with Adam on the mean squared error.
* **Control**: every T steps the network reads the current features; a
  greedy allocation starts every patch at the largest candidate and, while
  the predicted error of the window exceeds the window's share of the error
  budget, moves the patch with the best ratio of predicted error removed to
  bytes added to its next smaller candidate.  A patch whose predictions are
  not finite keeps the fixed threshold (the fallback).
* **Judge**: the fixed-threshold method, swept over the candidates; the
  learned run is compared with it at equal error (log-log interpolation of
  the sweep's compression ratio at the learned run's error).

Everything GPU-side runs through the C ABI of ``liblbmz``; this module holds
the bookkeeping and the allocation on the host.
"""
from __future__ import annotations

import argparse
import heapq
import json
import math
import sys
import time

import numpy as np

CANDIDATES = (1e-5, 3e-5, 1e-4, 3e-4, 1e-3, 3e-3)
K = len(CANDIDATES)
P = 64
LEVELS = 5
TAU = 0.6
WINDOW = 25
ERR_FLOOR = 1e-20


def _ctx(n, eps, reference=False):
    from .lbmz import Context
    return Context(n, scheme="d2q9_bgk", dtype="f32", p=P, wavelet="bl53", levels=LEVELS, eps=eps, tau=TAU,
                   reference=reference)


def _patch_sums(sq: np.ndarray, n: int) -> np.ndarray:
    """Per-patch sums of ``sq[9, n, n]`` in patch order (px + npx py)."""
    npx = n // P
    return sq.reshape(9, npx, P, npx, P).sum(axis=(0, 2, 4)).reshape(-1)


def _record_bytes(table: np.ndarray) -> np.ndarray:
    """Bytes of each patch's records (sum over fields), from the offset table."""
    from .lbmz import MASK_BIT
    nnz = (table[..., 1] & (MASK_BIT - 1)).astype(np.int64)
    is_mask = (table[..., 1] & MASK_BIT) != 0
    w = (65 * 65 + 63) // 64
    vb = (nnz * 4 + 7) // 8 * 8
    rb = (vb + np.where(is_mask, 8 * w, 2 * nnz) + 15) // 16 * 16
    return rb.sum(axis=1)


def snapshot_samples(n: int, seed: int, times, eps_run: float = 1e-4, window: int = WINDOW):
    """Network inputs and labels ``(x[B, 9, 8, 8], log10_err[B, K], log10_bytes[B, K])``."""
    from synth import shear_with_vortices
    rho, ux, uy = shear_with_vortices(n, seed=seed)
    macro = [a.astype(np.float32) for a in (rho, ux, uy)]
    run = _ctx(n, eps_run)
    run.enable_features(True)
    run.set_macroscopic(*macro)
    xs, es, bs = [], [], []
    t_done = 0
    for t in times:
        run.step(t - t_done)
        t_done = t
        feats = run.features().copy()
        table, pool = run.store()
        state = run.fields()
        ref = _ctx(n, 0.0, reference=True)
        for f in range(9):
            ref.set_field(f, state[f])
        ref.step(window)
        truth = ref.fields().astype(np.float64)
        ref.close()
        err = np.empty((feats.shape[0], K))
        byt = np.empty((feats.shape[0], K))
        for k, eps in enumerate(CANDIDATES):
            c = _ctx(n, eps)
            c.put_store(table, pool)
            c.step(window)
            d = c.fields().astype(np.float64) - truth
            err[:, k] = _patch_sums(d * d, n)
            byt[:, k] = _record_bytes(c.store()[0])
            c.close()
        xs.append(feats)
        es.append(np.log10(np.maximum(err, ERR_FLOOR)))
        bs.append(np.log10(byt))
    run.close()
    return np.concatenate(xs), np.concatenate(es), np.concatenate(bs)


def init_params(k_out: int, seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases, in the parameter order of include/lbmz.h."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in ((32, 9, 3, 3), (32,), (32, 32, 3, 3), (32,), (32, 32, 3, 3), (32,), (k_out, 32), (k_out,)):
        if len(shape) == 1:
            parts.append(np.zeros(shape))
        else:
            fan_in = int(np.prod(shape[1:]))
            lim = math.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, size=shape))
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


def train(x, y, epochs: int = 40, batch: int = 256, lr: float = 2e-3, seed: int = 0, val_frac: float = 0.1):
    """Train a network on ``x -> y``; returns ``(net, history)``."""
    from .lbmz import Net
    rng = np.random.default_rng(seed)
    nval = max(1, int(val_frac * x.shape[0]))
    perm = rng.permutation(x.shape[0])
    vi, ti = perm[:nval], perm[nval:]
    net = Net(y.shape[1])
    net.set_params(init_params(y.shape[1], seed))
    hist = []
    bs = min(batch, ti.size)
    for ep in range(epochs):
        order = rng.permutation(ti)
        losses = []
        for s in range(0, order.size - bs + 1, bs):
            b = order[s:s + bs]
            losses.append(net.train_step(x[b], y[b], lr))
        pv = net.forward(x[vi])
        hist.append({"epoch": ep, "train": float(np.mean(losses)), "val": float(np.mean((pv - y[vi]) ** 2))})
    return net, hist


def allocate(pred_err, pred_bytes, budget, fallback_index: int) -> np.ndarray:
    """Per-patch candidate index by the greedy allocation described above.

    A patch with any non-finite prediction is pinned to ``fallback_index`` and
    left out of both the predicted total and the budget, so that the finite
    patches are allocated exactly as they would be without it.  ``budget``
    None means the predicted error of the fallback threshold on the finite
    patches (the fixed method's own predicted error).
    """
    npatch = pred_err.shape[0]
    with np.errstate(over="ignore", invalid="ignore"):
        e = np.power(10.0, np.asarray(pred_err, dtype=np.float64))
        b = np.power(10.0, np.asarray(pred_bytes, dtype=np.float64))
    bad = ~(np.all(np.isfinite(e), axis=1) & np.all(np.isfinite(b), axis=1))
    good = np.flatnonzero(~bad)
    if budget is None:
        budget = float(np.sum(e[good, fallback_index]))
    idx = np.full(npatch, K - 1, dtype=np.int64)
    idx[bad] = fallback_index
    total = float(np.sum(e[good, K - 1]))
    heap = []

    def push(q):
        i = idx[q]
        if i == 0:
            return
        de = e[q, i] - e[q, i - 1]
        db = max(b[q, i - 1] - b[q, i], 1e-9)
        heapq.heappush(heap, (-(de / db), q, i))

    for q in good:
        push(q)
    while total > budget and heap:
        _, q, i = heapq.heappop(heap)
        if idx[q] != i:
            continue
        total -= e[q, i] - e[q, i - 1]
        idx[q] = i - 1
        push(q)
    return idx


def run_learned(net, n: int, seed: int, steps: int, fixed_eps: float, window: int = WINDOW):
    """The controlled run next to the uncompressed one; returns its summary.

    In every window the budget is the network's own predicted error of the
    fixed threshold ``fixed_eps`` on every patch: the allocation may only
    redistribute the thresholds so that the predicted error of the window
    stays at most that of the fixed method, and saves bytes where it can.
    ``fixed_eps`` is also the fallback of a patch without finite predictions.
    """
    from synth import shear_with_vortices
    rho, ux, uy = shear_with_vortices(n, seed=seed)
    macro = [a.astype(np.float32) for a in (rho, ux, uy)]
    ref = _ctx(n, 0.0, reference=True)
    ref.set_macroscopic(*macro)
    ref.step(steps)
    truth = ref.fields().astype(np.float64)
    ref.close()
    fb = CANDIDATES.index(fixed_eps)
    c = _ctx(n, fixed_eps)
    c.enable_features(True)
    c.set_macroscopic(*macro)
    c.step(1)
    done, ratios, chosen = 1, [], []
    t0 = time.perf_counter()
    while done < steps:
        pred = net.forward(c.features())
        pe, pb = pred[:, :K], pred[:, K:]
        idx = allocate(pe, pb, None, fb)
        c.set_patch_eps(np.array([CANDIDATES[i] for i in idx], dtype=np.float64))
        chosen.append(np.bincount(idx, minlength=K).tolist())
        w = min(window, steps - done)
        c.step(w)
        done += w
        ratios.append(c.stats()["ratio"])
    wall = time.perf_counter() - t0
    sim = c.fields().astype(np.float64)
    c.close()
    return {"rel_l2": float(np.linalg.norm(sim - truth) / np.linalg.norm(truth)),
            "ratio_mean": float(np.mean(ratios)), "ratio_final": float(ratios[-1]),
            "choices": np.sum(np.array(chosen), axis=0).tolist(), "seconds": wall}


def fixed_sweep(n: int, seed: int, steps: int, window: int = WINDOW):
    """The judge: every candidate as a fixed threshold (ratio averaged like the learned run's)."""
    from synth import shear_with_vortices
    rho, ux, uy = shear_with_vortices(n, seed=seed)
    macro = [a.astype(np.float32) for a in (rho, ux, uy)]
    ref = _ctx(n, 0.0, reference=True)
    ref.set_macroscopic(*macro)
    ref.step(steps)
    truth = ref.fields().astype(np.float64)
    ref.close()
    out = []
    for eps in CANDIDATES:
        c = _ctx(n, eps)
        c.set_macroscopic(*macro)
        c.step(1)
        done, ratios = 1, []
        while done < steps:
            w = min(window, steps - done)
            c.step(w)
            done += w
            ratios.append(c.stats()["ratio"])
        sim = c.fields().astype(np.float64)
        c.close()
        out.append({"eps": eps, "rel_l2": float(np.linalg.norm(sim - truth) / np.linalg.norm(truth)),
                    "ratio_mean": float(np.mean(ratios))})
    return out


def ratio_at_error(sweep, err: float):
    """Log-log interpolation of the fixed sweep's mean ratio at a relative L2 error."""
    pts = sorted((p["rel_l2"], p["ratio_mean"]) for p in sweep if p["rel_l2"] > 0)
    for (e0, r0), (e1, r1) in zip(pts, pts[1:]):
        if e0 <= err <= e1 and e1 > e0:
            w = (math.log(err) - math.log(e0)) / (math.log(e1) - math.log(e0))
            return math.exp(math.log(r0) + w * (math.log(r1) - math.log(r0)))
    return None


def evaluate(n_train: int = 512, train_seeds=(1, 2, 3, 4, 5, 6), times=(50, 150, 250, 350),
             n_eval: int = 1024, eval_seed: int = 100, steps: int = 500, fixed=(1e-5, 3e-5, 1e-4),
             epochs: int = 40):
    """Data, training, the fixed sweep and one controlled run per fixed
    threshold it is measured against; returns a summary."""
    t0 = time.perf_counter()
    xs, es, bs = [], [], []
    for s in train_seeds:
        x, e, b = snapshot_samples(n_train, s, times)
        xs.append(x)
        es.append(e)
        bs.append(b)
    x = np.concatenate(xs)
    y = np.concatenate([np.concatenate(es), np.concatenate(bs)], axis=1).astype(np.float32)
    t_data = time.perf_counter() - t0
    net, hist = train(x, y, epochs=epochs)
    t_train = time.perf_counter() - t0 - t_data
    sweep = fixed_sweep(n_eval, eval_seed, steps)
    runs = []
    for eps in fixed:
        learned = run_learned(net, n_eval, eval_seed, steps, eps)
        same = ratio_at_error(sweep, learned["rel_l2"])
        base = next(p for p in sweep if p["eps"] == eps)
        runs.append({"fixed_eps": eps, "fixed_rel_l2": base["rel_l2"], "fixed_ratio": base["ratio_mean"],
                     "learned": learned, "fixed_ratio_at_learned_error": same,
                     "gain": (learned["ratio_mean"] / same) if same else None})
    net.close()
    return {"samples": int(x.shape[0]), "data_seconds": t_data, "train_seconds": t_train, "history": hist[-3:],
            "fixed": sweep, "runs": runs,
            "config": {"n_train": n_train, "train_seeds": list(train_seeds), "times": list(times),
                       "n_eval": n_eval, "eval_seed": eval_seed, "steps": steps, "window": WINDOW,
                       "candidates": list(CANDIDATES)}}


def main(argv=None):
    ap = argparse.ArgumentParser(description="learned per-patch thresholds vs fixed eps (GPU)")
    ap.add_argument("--n-train", type=int, default=512)
    ap.add_argument("--n-eval", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--fixed", type=float, nargs="*", default=[1e-5, 3e-5, 1e-4],
                    help="fixed thresholds the controlled runs are measured against")
    ap.add_argument("--train-seeds", type=int, default=6, help="training runs use seeds 1..N")
    ap.add_argument("--times", type=int, nargs="*", default=[50, 150, 250, 350],
                    help="steps at which each training run is stopped for samples")
    ap.add_argument("--json", default=None)
    args = ap.parse_args(argv)
    res = evaluate(n_train=args.n_train, train_seeds=tuple(range(1, args.train_seeds + 1)), times=tuple(args.times),
                   n_eval=args.n_eval, steps=args.steps, epochs=args.epochs, fixed=tuple(args.fixed))
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(res, fh, indent=1)
    print(f"samples {res['samples']}  data {res['data_seconds']:.1f} s  training {res['train_seconds']:.1f} s  "
          f"last losses {res['history'][-1]}")
    for p in res["fixed"]:
        print(f"  fixed eps {p['eps']:.0e}: rel_l2 {p['rel_l2']:.3e}  mean ratio {p['ratio_mean']:.1f}")
    for r in res["runs"]:
        L = r["learned"]
        print(f"  against eps {r['fixed_eps']:.0e}: learned rel_l2 {L['rel_l2']:.3e}  mean ratio {L['ratio_mean']:.1f}"
              f"  choices {L['choices']}  fixed ratio at that error {r['fixed_ratio_at_learned_error']}"
              f"  gain {r['gain']}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
