"""Reduced-precision coefficient storage on the compressible-Euler workload (GPU).

Workload: the compressible Euler equations with the first-order Rusanov flux
(four conserved fields, float32 stencil arithmetic) on a 4096 x 4096
periodic grid in 64 x 64 patches (folded BL5/3, 5 levels, capped threshold),
from a seeded four-quadrant Riemann problem (density and pressure uniform in
[0.1, 1.5], gas at rest), 500 steps.  The coefficients are stored as float32,
or as float32 samples plus binary16 / E4M3 details with per-subband
power-of-two scales; the conserved totals are reduced in float64.

For each value format it reports the throughput (cell updates per second of
the whole compressed step, HIP events), the compression ratio, the error
against the uncompressed float32 run of the same scheme (relative L2 and
L-infinity over the four fields, and the paper's equation "L2_error" on the
density), and the drift of the four conserved totals.

Readings: the time step is dt = CFL h / s_max with CFL = 0.4 and s_max twice
the largest initial sound speed (the gas starts at rest; the factor bounds
the wave speeds the Riemann fans reach); gamma = 1.4; eps = 1e-4.

Everything runs through the C ABI of ``liblbmz``; this module loops over the
formats and does the bookkeeping on the host.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

N = 4096
PATCH = 64
LEVELS = 5
EPS = 1e-4
STEPS = 500
GAMMA = 1.4
CFL = 0.4
SEED = 0
FORMATS = ("f32", "f16", "e4m3", "e4m3b")


def problem(n: int = N, seed: int = SEED):
    from synth import riemann_four_quadrants
    w, states = riemann_four_quadrants(n, seed=seed, gamma=GAMMA)
    smax = 2.0 * max(np.sqrt(GAMMA * p / r) for r, p in states)
    return w.astype(np.float32), smax


def _ctx(n, smax, values="f32", reference=False, eps=EPS, levels=LEVELS, p=PATCH):
    from .lbmz import Context
    return Context(n, scheme="euler_rusanov", dtype="f32", p=p, wavelet="bl53", levels=levels, eps=eps,
                   vel=(smax, 0.0), cfl=CFL, gamma=GAMMA, values=values, reference=reference)


def _set(ctx, w):
    for f in range(4):
        ctx.set_field(f, w[f])


def run(n: int = N, steps: int = STEPS, formats=FORMATS, eps: float = EPS, warmup: int = 5):
    """All formats against the uncompressed run; returns a result dict."""
    import torch

    w, smax = problem(n)
    ref = _ctx(n, smax, reference=True)
    _set(ref, w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref.step(warmup + steps)
    torch.cuda.synchronize()
    ref_s = time.perf_counter() - t0
    plain = ref.fields().astype(np.float64)
    ref.close()
    h = 1.0 / n
    out = {"grid": n, "patch": PATCH, "levels": LEVELS, "eps": eps, "steps": steps, "warmup": warmup,
           "cfl": CFL, "gamma": GAMMA, "s_max": smax,
           "uncompressed_mlups": n * n * (warmup + steps) / ref_s / 1e6, "formats": []}
    from .lbmz import LBMZ_ENAN, LbmzError
    for v in formats:
        ctx = _ctx(n, smax, values=v, eps=eps)
        _set(ctx, w)
        t0 = np.array(ctx.stats()["totals"])
        try:
            ctx.step(warmup)
            torch.cuda.synchronize()
            a = time.perf_counter()
            ctx.step(steps)
            torch.cuda.synchronize()
        except LbmzError as e:
            if e.code != LBMZ_ENAN:
                raise
            st = ctx.stats()
            ctx.close()
            out["formats"].append({"values": v, "failed": "non-finite state (negative density or pressure)",
                                   "steps_done": int(st["steps"]), "ratio": st["ratio"]})
            continue
        wall = time.perf_counter() - a
        st = ctx.stats()
        sim = ctx.fields().astype(np.float64)
        ctx.close()
        d = sim - plain
        t1 = np.array(st["totals"])
        out["formats"].append({
            "values": v,
            "mlups": n * n * steps / wall / 1e6,
            "mlups_events": n * n * steps / (st["ms_last_call"] * 1e-3) / 1e6,
            "kernel_ms_avg": st["ms_last_call"] / steps,
            "ratio": st["ratio"],
            "store_bytes": st["store_bytes"],
            "rel_l2": float(np.linalg.norm(d) / np.linalg.norm(plain)),
            "linf": float(np.max(np.abs(d))),
            "paper_l2_density": float(h * h * np.sum(d[0] ** 2)),
            "totals_drift": [float(x) for x in (t1 - t0)],
            "totals_rel": [float(abs(x) / max(abs(y), 1e-30)) for x, y in zip(t1 - t0, t0)],
        })
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="reduced-precision storage on the Euler workload (GPU)")
    ap.add_argument("--n", type=int, default=N)
    ap.add_argument("--steps", type=int, default=STEPS)
    ap.add_argument("--eps", type=float, default=EPS)
    ap.add_argument("--json", default=None)
    args = ap.parse_args(argv)
    res = run(args.n, args.steps, eps=args.eps)
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(res, fh, indent=1)
    print(f"Euler Rusanov {res['grid']}^2, {res['steps']} steps, eps {res['eps']}; "
          f"uncompressed {res['uncompressed_mlups']:.0f} MLUPS")
    for r in res["formats"]:
        if "failed" in r:
            print(f"  {r['values']:5s} stopped after {r['steps_done']} steps: {r['failed']}")
            continue
        print(f"  {r['values']:5s} {r['mlups_events']:9.0f} MLUPS  ratio {r['ratio']:8.2f}  "
              f"rel_l2 {r['rel_l2']:.3e}  linf {r['linf']:.3e}  mass drift {r['totals_rel'][0]:.1e}  "
              f"energy drift {r['totals_rel'][3]:.1e}")
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
