"""Execution modes of the step on the two hot-path workloads (GPU).

For each workload the autotuner of the library times the four modes -- one
workgroup per patch or a persistent work-queue kernel, plain launches or HIP
graph chunks -- on the real state (the modes compute identical records) and
keeps the fastest.  Workloads: the 256^2 upwind-transport run (64 patches of
32^2, Haar, 4 levels, float64: launch-bound) and the 2048^2 D2Q9 run (1024
patches of 64^2, BL5/3, 5 levels, float32).
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np


def measure(steps_per_variant: int = 10):
    from synth import fv_gaussians_and_step, shear_layer_macroscopic

    from .lbmz import Context

    out = {}
    c = Context(256, scheme="fv_upwind", dtype="f64", p=32, wavelet="haar", levels=4, eps=1e-4)
    c.set_field(0, fv_gaussians_and_step(256, seed=0))
    ms = c.autotune(steps_per_variant)
    out["transport_256_f64"] = {"ms_per_step": [float(v) for v in ms], "chosen": c.execution()}
    c.close()
    n = 2048
    c = Context(n, scheme="d2q9_bgk", dtype="f32", p=64, wavelet="bl53", levels=5, eps=1e-4, tau=0.6)
    rho, ux, uy = shear_layer_macroscopic(n, seed=0)
    c.set_macroscopic(*(a.astype(np.float32) for a in (rho, ux, uy)))
    ms = c.autotune(steps_per_variant)
    out["d2q9_2048_f32"] = {"ms_per_step": [float(v) for v in ms], "chosen": c.execution()}
    c.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="execution modes of the step (GPU)")
    ap.add_argument("--steps", type=int, default=10)
    args = ap.parse_args(argv)
    res = measure(args.steps)
    names = ("plain", "graph", "persistent", "persistent+graph")
    for w, r in res.items():
        cells = "  ".join(f"{nm} {1e3 * v:8.2f} us" for nm, v in zip(names, r["ms_per_step"]))
        print(f"{w:20s} {cells}   chosen persistent={r['chosen'][0]} graph={r['chosen'][1]}")
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
