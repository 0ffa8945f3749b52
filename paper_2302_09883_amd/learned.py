"""Learned per-patch threshold controls on the D2Q9 workload (GPU).

The paper sets one threshold constant and one compression level per run by
hand for an error target (Section 2.2, Section 3.2).  Here a small network
chooses both per patch, and the fixed-threshold method is its fallback and
its judge:

* **Controls.**  A candidate is a pair (threshold constant eps, threshold
  level count L_t): the L_t finest detail levels of the patch may be zeroed
  (``Context.set_patch_eps`` / ``set_patch_levels``; shared bordering lines
  take the smaller threshold of their tiles, which keeps the shared values
  and the conservation of the totals).
* **Data** from the plain method's own runs: a compressed D2Q9 run (double
  shear layer plus seeded vortices) is stopped at several times; from each
  stopped state, every candidate is run for a window of T steps next to the
  uncompressed scheme started from the same decompressed state.  Per patch:
  the network input of the stopped state (``Context.features``: the stored
  coefficients at stride 8 and the energies of the three finest levels per
  8 x 8 block), and per candidate the log10 squared error the window added in
  the patch and the log10 bytes of the patch's records.
* **Network** (``Net``, hand-written HIP kernels, bfloat16 weights): features
  -> 2 K outputs, trained with Adam on the mean squared error.
* **Control.**  Every T steps the network reads the current features; a
  greedy allocation on each patch's lower convex hull of predicted (bytes,
  error) starts every patch at its fewest bytes and, while the predicted
  error of the window exceeds the network's own prediction for the fixed
  candidate on every patch, moves the patch with the most predicted error
  removed per byte added one hull point further.  A patch whose predictions
  are not finite keeps the fixed candidate (the fallback).
* **Judge.**  Each window also runs, from the same state, the fixed
  threshold on every patch and the uncompressed scheme; the learned window is
  kept only if it adds no more squared error than the fixed window and its
  store is no larger, otherwise the fixed window's state replaces it.

Everything GPU-side runs through the C ABI of ``liblbmz``; error sums are
taken on the device with PyTorch tensors (measurement), the allocation on the
host.
"""
from __future__ import annotations

import argparse
import heapq
import json
import math
import sys
import time

import numpy as np

EPS = (3e-6, 1e-5, 3e-5, 1e-4, 3e-4)
LEVS = (5, 4, 3)                       # threshold level counts (5 = every detail level)
CANDIDATES = tuple((e, lv) for e in EPS for lv in LEVS)
K = len(CANDIDATES)
P = 64
LEVELS = 5
TAU = 0.6
WINDOW = 25
ERR_FLOOR = 1e-30


def _say(msg: str):
    print("[learned]", msg, file=sys.stderr, flush=True)


def candidate_index(eps: float, lev: int = LEVELS) -> int:
    return CANDIDATES.index((eps, lev))


def _ctx(n, eps, reference=False):
    from .lbmz import Context
    return Context(n, scheme="d2q9_bgk", dtype="f32", p=P, wavelet="bl53", levels=LEVELS, eps=eps, tau=TAU,
                   reference=reference)


def _set_controls(ctx, idx):
    """Per-patch eps and threshold level counts of candidate indices ``idx``."""
    ctx.set_patch_eps(np.array([CANDIDATES[i][0] for i in idx], dtype=np.float64))
    ctx.set_patch_levels(np.array([CANDIDATES[i][1] for i in idx], dtype=np.int32))


def _record_bytes(table: np.ndarray) -> np.ndarray:
    """Bytes of each patch's records (sum over fields), from the offset table."""
    from .lbmz import MASK_BIT
    nnz = (table[..., 1] & (MASK_BIT - 1)).astype(np.int64)
    is_mask = (table[..., 1] & MASK_BIT) != 0
    w = (65 * 65 + 63) // 64
    vb = (nnz * 4 + 7) // 8 * 8
    rb = (vb + np.where(is_mask, 8 * w, 2 * nnz) + 15) // 16 * 16
    return rb.sum(axis=1)


class _Fields:
    """Device copies of a context's fields (PyTorch float32 tensors)."""

    def __init__(self, n):
        import torch
        self.t = torch.empty((9, n, n), dtype=torch.float32, device="cuda")

    def read(self, ctx):
        for f in range(9):
            ctx.decompress_field(f, out=self.t[f])
        return self.t

    def write(self, ctx):
        for f in range(9):
            ctx.set_field(f, self.t[f])


def _patch_sq_errors(a, b, n):
    """Per-patch sums of squared differences of two [9, n, n] tensors (float64, host)."""
    d = (a.double() - b.double()) ** 2
    npx = n // P
    return d.reshape(9, npx, P, npx, P).sum(dim=(0, 2, 4)).reshape(-1).cpu().numpy()


def snapshot_samples(n: int, seed: int, times, eps_run: float = 1e-4, window: int = WINDOW):
    """Network inputs and labels ``(x[B, 36, 8, 8], log10_err[B, K], log10_bytes[B, K])``."""
    from synth import shear_with_vortices
    rho, ux, uy = shear_with_vortices(n, seed=seed)
    macro = [a.astype(np.float32) for a in (rho, ux, uy)]
    run = _ctx(n, eps_run)
    run.enable_features(True)
    run.set_macroscopic(*macro)
    ref = _ctx(n, 0.0, reference=True)
    cands = {e: _ctx(n, e) for e in EPS}
    buf, truth = _Fields(n), _Fields(n)
    xs, es, bs = [], [], []
    t_done = 0
    for t in times:
        run.step(t - t_done)
        t_done = t
        feats = run.features().copy()
        table, pool = run.store()
        buf.read(run)
        buf.write(ref)
        ref.step(window)
        tt = truth.read(ref)
        err = np.empty((feats.shape[0], K))
        byt = np.empty((feats.shape[0], K))
        for k, (eps, lev) in enumerate(CANDIDATES):
            c = cands[eps]
            c.set_patch_levels(np.full(feats.shape[0], lev, dtype=np.int32))
            c.put_store(table, pool)
            c.step(window)
            err[:, k] = _patch_sq_errors(buf.read(c), tt, n)
            byt[:, k] = _record_bytes(c.store()[0])
        xs.append(feats)
        es.append(np.log10(np.maximum(err, ERR_FLOOR)))
        bs.append(np.log10(byt))
    for c in cands.values():
        c.close()
    ref.close()
    run.close()
    return np.concatenate(xs), np.concatenate(es), np.concatenate(bs)


def init_params(k_out: int, seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases, in the parameter order of include/lbmz.h."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in ((32, 12, 3, 3), (32,), (32, 32, 3, 3), (32,), (32, 32, 3, 3), (32,), (k_out, 32), (k_out,)):
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
        if ep % 5 == 0:
            _say(f"epoch {ep}")
        order = rng.permutation(ti)
        losses = []
        for s in range(0, order.size - bs + 1, bs):
            b = order[s:s + bs]
            losses.append(net.train_step(x[b], y[b], lr))
        pv = net.forward(x[vi])
        hist.append({"epoch": ep, "train": float(np.mean(losses)), "val": float(np.mean((pv - y[vi]) ** 2))})
    return net, hist


def _hull(e, b):
    """Candidate indices of one patch's lower convex hull of (bytes, error),
    from the fewest bytes on, each next point the one removing the most error
    per byte added."""
    order = sorted(range(len(e)), key=lambda k: (b[k], e[k]))
    chain = [order[0]]
    while True:
        cur = chain[-1]
        best, slope = None, 0.0
        for k in order:
            if b[k] > b[cur] and e[k] < e[cur]:
                s = (e[k] - e[cur]) / (b[k] - b[cur])
                if best is None or s < slope:
                    best, slope = k, s
        if best is None:
            return chain
        chain.append(best)


def allocate(pred_err, pred_bytes, budget, fallback_index: int) -> np.ndarray:
    """Per-patch candidate index by the greedy allocation described above.

    A patch with any non-finite prediction is pinned to ``fallback_index`` and
    left out of both the predicted total and the budget, so that the finite
    patches are allocated exactly as they would be without it.  ``budget``
    None means the predicted error of the fallback candidate on the finite
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
    idx = np.full(npatch, fallback_index, dtype=np.int64)
    chains, pos = {}, {}
    total = 0.0
    heap = []
    for q in good:
        ch = _hull(e[q], b[q])
        chains[q], pos[q] = ch, 0
        idx[q] = ch[0]
        total += e[q, ch[0]]
        if len(ch) > 1:
            k0, k1 = ch[0], ch[1]
            heapq.heappush(heap, ((e[q, k1] - e[q, k0]) / (b[q, k1] - b[q, k0]), int(q)))
    while total > budget and heap:
        _, q = heapq.heappop(heap)
        ch, i = chains[q], pos[q]
        k0, k1 = ch[i], ch[i + 1]
        total += e[q, k1] - e[q, k0]
        pos[q] = i + 1
        idx[q] = k1
        if i + 2 < len(ch):
            k2 = ch[i + 2]
            heapq.heappush(heap, ((e[q, k2] - e[q, k1]) / (b[q, k2] - b[q, k1]), int(q)))
    return idx


def _truth_run(n, macro, steps):
    ref = _ctx(n, 0.0, reference=True)
    ref.set_macroscopic(*macro)
    ref.step(steps)
    out = _Fields(n)
    t = out.read(ref).clone()
    ref.close()
    return t


def _rel_l2(a, b):
    return float(((a.double() - b.double()) ** 2).sum().sqrt() / (b.double() ** 2).sum().sqrt())


def run_learned(net, n: int, seed: int, steps: int, fixed_eps: float, window: int = WINDOW, judge: bool = True):
    """The controlled run; returns its summary (error against the
    uncompressed run of the same length, mean ratio, choices, judge record)."""
    from synth import shear_with_vortices
    rho, ux, uy = shear_with_vortices(n, seed=seed)
    macro = [a.astype(np.float32) for a in (rho, ux, uy)]
    truth = _truth_run(n, macro, steps)
    fb = candidate_index(fixed_eps)
    a = _ctx(n, fixed_eps)
    a.enable_features(True)
    a.set_macroscopic(*macro)
    a.step(1)
    b = r = None
    buf, tw = _Fields(n), _Fields(n)
    if judge:
        b = _ctx(n, fixed_eps)
        b.enable_features(True)
        r = _ctx(n, 0.0, reference=True)
    done, ratios, chosen, kept, feats = 1, [], [], [], a.features()
    t0 = time.perf_counter()
    while done < steps:
        pred = net.forward(feats)
        idx = allocate(pred[:, :K], pred[:, K:], None, fb)
        chosen.append(np.bincount(idx, minlength=K).tolist())
        w = min(window, steps - done)
        if judge:
            table, pool = a.store()
            b.put_store(table, pool)
            buf.read(a)
            buf.write(r)
        _set_controls(a, idx)
        a.step(w)
        ok = True
        if judge:
            b.step(w)
            r.step(w)
            tt = tw.read(r)
            ea = float(((buf.read(a).double() - tt.double()) ** 2).sum())
            eb = float(((buf.read(b).double() - tt.double()) ** 2).sum())
            ok = ea <= eb and a.stats()["store_bytes"] <= b.stats()["store_bytes"]
            if not ok:
                table, pool = b.store()
                a.put_store(table, pool)
        kept.append(ok)
        feats = a.features() if ok else b.features()
        done += w
        ratios.append(a.stats()["ratio"])
    wall = time.perf_counter() - t0
    sim = buf.read(a)
    out = {"rel_l2": _rel_l2(sim, truth), "ratio_mean": float(np.mean(ratios)), "ratio_final": float(ratios[-1]),
           "choices": np.sum(np.array(chosen), axis=0).tolist(), "windows": len(kept),
           "windows_kept": int(np.sum(kept)), "seconds": wall}
    for c in (a, b, r):
        if c is not None:
            c.close()
    return out


def fixed_sweep(n: int, seed: int, steps: int, window: int = WINDOW, eps_list=EPS):
    """The fixed method: every candidate threshold on every patch (ratio
    averaged over the same window ends as the controlled run's)."""
    from synth import shear_with_vortices
    rho, ux, uy = shear_with_vortices(n, seed=seed)
    macro = [a.astype(np.float32) for a in (rho, ux, uy)]
    truth = _truth_run(n, macro, steps)
    buf = _Fields(n)
    out = []
    for eps in eps_list:
        c = _ctx(n, eps)
        c.set_macroscopic(*macro)
        c.step(1)
        done, ratios = 1, []
        while done < steps:
            w = min(window, steps - done)
            c.step(w)
            done += w
            ratios.append(c.stats()["ratio"])
        out.append({"eps": eps, "rel_l2": _rel_l2(buf.read(c), truth), "ratio_mean": float(np.mean(ratios))})
        c.close()
    return out


def ratio_at_error(sweep, err: float):
    """Log-log interpolation of the fixed sweep's mean ratio at a relative L2
    error (None outside the swept errors)."""
    pts = sorted((p["rel_l2"], p["ratio_mean"]) for p in sweep if p["rel_l2"] > 0)
    for (e0, r0), (e1, r1) in zip(pts, pts[1:]):
        if e0 <= err <= e1 and e1 > e0:
            w = (math.log(err) - math.log(e0)) / (math.log(e1) - math.log(e0))
            return math.exp(math.log(r0) + w * (math.log(r1) - math.log(r0)))
    return None


def evaluate(n_train: int = 512, train_seeds=(1, 2, 3, 4, 5, 6), times=(50, 150, 250, 350),
             n_eval: int = 1024, eval_seed: int = 100, steps: int = 500, fixed=(3e-6, 1e-5, 3e-5, 1e-4),
             epochs: int = 40, budget: float = 1e-3, judge: bool = True):
    """Data, training, the fixed sweep and one controlled run per fixed
    threshold it is measured against; returns a summary."""
    t0 = time.perf_counter()
    xs, es, bs = [], [], []
    for i, s in enumerate(train_seeds):
        x, e, b = snapshot_samples(n_train, s, times, eps_run=EPS[i % len(EPS)])
        xs.append(x)
        es.append(e)
        bs.append(b)
        _say(f"training data: seed {s} done, {sum(a.shape[0] for a in xs)} samples")
    x = np.concatenate(xs)
    y = np.concatenate([np.concatenate(es), np.concatenate(bs)], axis=1).astype(np.float32)
    t_data = time.perf_counter() - t0
    del xs
    net, hist = train(x, y, epochs=epochs)
    t_train = time.perf_counter() - t0 - t_data
    _say(f"trained: {hist[-1]}")
    sweep = fixed_sweep(n_eval, eval_seed, steps)
    _say("fixed sweep: " + ", ".join(f"{p['eps']:.0e}: {p['rel_l2']:.3e} / {p['ratio_mean']:.1f}" for p in sweep))
    # the error budget: the best fixed threshold meeting it is also a reference of a controlled run
    meet = [p for p in sweep if p["rel_l2"] <= budget]
    best = max(meet, key=lambda p: p["ratio_mean"]) if meet else None
    if best is not None and best["eps"] not in fixed:
        fixed = tuple(fixed) + (best["eps"],)
    runs = []
    for eps in fixed:
        learned = run_learned(net, n_eval, eval_seed, steps, eps, judge=judge)
        _say(f"controlled run against eps {eps:.0e}: {learned}")
        same = ratio_at_error(sweep, learned["rel_l2"])
        base = next(p for p in sweep if p["eps"] == eps)
        runs.append({"fixed_eps": eps, "fixed_rel_l2": base["rel_l2"], "fixed_ratio": base["ratio_mean"],
                     "learned": learned, "fixed_ratio_at_learned_error": same,
                     "gain": (learned["ratio_mean"] / same) if same else None,
                     "ratio_gain_over_fixed": learned["ratio_mean"] / base["ratio_mean"]})
    at_budget = None
    if best is not None:
        r = next((r for r in runs if r["fixed_eps"] == best["eps"]), None)
        at_budget = {"budget": budget, "fixed_eps": best["eps"], "fixed_ratio": best["ratio_mean"],
                     "learned_ratio": r["learned"]["ratio_mean"] if r else None,
                     "learned_rel_l2": r["learned"]["rel_l2"] if r else None}
    net.close()
    return {"samples": int(x.shape[0]), "data_seconds": t_data, "train_seconds": t_train, "history": hist[-3:],
            "fixed": sweep, "runs": runs, "at_budget": at_budget,
            "config": {"n_train": n_train, "train_seeds": list(train_seeds), "times": list(times),
                       "n_eval": n_eval, "eval_seed": eval_seed, "steps": steps, "window": WINDOW,
                       "candidates": [list(c) for c in CANDIDATES], "judge": judge}}


def main(argv=None):
    ap = argparse.ArgumentParser(description="learned per-patch threshold controls vs fixed eps (GPU)")
    ap.add_argument("--n-train", type=int, default=512)
    ap.add_argument("--n-eval", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--fixed", type=float, nargs="*", default=[3e-6, 1e-5, 3e-5, 1e-4],
                    help="fixed thresholds the controlled runs are measured against")
    ap.add_argument("--train-seeds", type=int, default=6, help="training runs use seeds 1..N")
    ap.add_argument("--times", type=int, nargs="*", default=[50, 150, 250, 350],
                    help="steps at which each training run is stopped for samples")
    ap.add_argument("--budget", type=float, default=1e-3)
    ap.add_argument("--no-judge", action="store_true", help="controlled runs without the fixed-window judge")
    ap.add_argument("--json", default=None)
    args = ap.parse_args(argv)
    res = evaluate(n_train=args.n_train, train_seeds=tuple(range(1, args.train_seeds + 1)), times=tuple(args.times),
                   n_eval=args.n_eval, steps=args.steps, epochs=args.epochs, fixed=tuple(args.fixed),
                   budget=args.budget, judge=not args.no_judge)
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
              f"  windows kept {L['windows_kept']}/{L['windows']}  fixed ratio at that error "
              f"{r['fixed_ratio_at_learned_error']}  gain {r['gain']}")
    print("  at budget:", res["at_budget"])
    return 0


if __name__ == "__main__":
    sys.exit(main())
